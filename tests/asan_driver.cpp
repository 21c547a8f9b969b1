// Host-only driver for the sanitizer check: the CPU oracle, the seeded input
// generator and the C ABI's argument validation, built together with
// AddressSanitizer and UndefinedBehaviorSanitizer (no GPU, no Python). It runs
// every function of the three over inputs that reach their edge cases --
// 3x3 views, ragged and downsampled views, empty selections, a capacity
// overflow, feature rows, invalid ABI arguments -- and checks a few results
// the paper's definitions fix (closed forms also pinned by the Python tests),
// so that a run that completes is also a run that computed something.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../paper_2603_08661_amd/csrc/validate.h"

extern "C" {
// oracle/igsp_oracle.c
void orc_blur_taps(int64_t* out5);
int32_t orc_bin(int64_t gx, int64_t gy);
void orc_nms(const int64_t* gx, const int64_t* gy, int32_t W, int32_t H, int64_t* M, uint8_t* bin, uint8_t* keep,
             double* margin);
int64_t orc_edge_view(const uint8_t* rgb, int32_t W, int32_t H, int64_t* gray_o, int64_t* b_o, int64_t* gx_o,
                      int64_t* gy_o, int64_t* M_o, uint8_t* bin_o, uint8_t* keep_o, double* m_o, double* E,
                      double* margin_o, double* med_o, int64_t* Mmed_o);
void orc_edge_batch(const uint8_t* rgb, int32_t n, const int32_t* W, const int32_t* H, const int64_t* in_off,
                    const int64_t* out_off, double* E, uint8_t* keep_out, double* med_out, int64_t* nsurv_out,
                    int32_t threads);
void orc_quat_to_R(const double q_in[4], double R[9]);
double orc_opacity(double o, double beta);
int32_t orc_las(int64_t N, int64_t capacity, const float* means, const float* log_scales, const float* quats,
                const float* opac, const float* feats, int32_t F, const uint8_t* mask, double alpha, double gamma,
                double beta, double* means_o, double* ls_o, double* quats_o, double* opac_o, double* feats_o,
                int32_t* split_idx, int32_t* axis, int64_t* K_out, int64_t* count_out);
// synth/synth.c
void syn_image(uint64_t seed, int32_t W, int32_t H, int32_t n_poly, int32_t texture, double tex_amp,
               double noise_sigma, uint8_t* out);
void syn_image_down2(uint64_t seed, int32_t W, int32_t H, int32_t n_poly, int32_t texture, double tex_amp,
                     double noise_sigma, uint8_t* out);
void syn_image_batch(int32_t n, const uint64_t* seeds, const int32_t* fw, const int32_t* fh, const int32_t* down2,
                     int32_t n_poly, int32_t texture, double tex_amp, double noise_sigma, const int64_t* offsets,
                     uint8_t* out);
void syn_view_sizes(uint64_t seed, int32_t n, int32_t wlo, int32_t whi, double alo, double ahi, int32_t* W,
                    int32_t* H);
void syn_gaussians(uint64_t seed, int64_t N, double ls_mu, double ls_sd, float* means, float* log_scales,
                   float* quats, float* opacity);
void syn_mask(uint64_t seed, int64_t N, int64_t K, uint8_t* mask);
int64_t syn_contrib_count(uint64_t seed, int64_t n_gauss, int32_t n_views, const int32_t* W, const int32_t* H,
                          int32_t mean_radius, int64_t* offsets);
void syn_contrib_fill(uint64_t seed, int64_t n_gauss, int32_t n_views, const int32_t* W, const int32_t* H,
                      int32_t mean_radius, const int64_t* offsets, int32_t order, int32_t* gauss, int32_t* view,
                      int32_t* pixel, float* weight);
}

static int g_fail = 0;
#define CHECK(c)                                                      \
  do {                                                                \
    if (!(c)) {                                                       \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      ++g_fail;                                                       \
    }                                                                 \
  } while (0)

// Every stage of one view, with every optional output requested.
static int64_t edge_all(const uint8_t* rgb, int W, int H, std::vector<double>* E_out = nullptr,
                        std::vector<uint8_t>* keep_out = nullptr, std::vector<int64_t>* gx_out = nullptr) {
  const size_t n = (size_t)W * H;
  std::vector<int64_t> gray(n), b(n), gx(n), gy(n), M(n);
  std::vector<uint8_t> bin(n), keep(n);
  std::vector<double> m(n), E(n), margin(n);
  double med = -1.0;
  int64_t Mmed = -1;
  const int64_t ns = orc_edge_view(rgb, W, H, gray.data(), b.data(), gx.data(), gy.data(), M.data(), bin.data(),
                                   keep.data(), m.data(), E.data(), margin.data(), &med, &Mmed);
  // the same view with no optional output at all
  std::vector<double> E2(n);
  CHECK(orc_edge_view(rgb, W, H, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                      E2.data(), nullptr, nullptr, nullptr) == ns);
  CHECK(std::memcmp(E.data(), E2.data(), n * sizeof(double)) == 0);
  if (E_out) *E_out = E;
  if (keep_out) *keep_out = keep;
  if (gx_out) *gx_out = gx;
  return ns;
}

static void edge_checks() {
  int64_t taps[5];
  orc_blur_taps(taps);
  CHECK(taps[0] == 1 && taps[1] == 4 && taps[2] == 6 && taps[3] == 4 && taps[4] == 1);
  CHECK(orc_bin(5, 1) == 0 && orc_bin(1, 5) == 1 && orc_bin(3, 3) == 2 && orc_bin(3, -3) == 3 && orc_bin(0, 0) == 3);
  // synthetic views of many shapes, including the smallest allowed
  const int sizes[][2] = {{3, 3}, {4, 3}, {3, 7}, {17, 5}, {37, 29}, {256, 192}, {301, 17}};
  for (const auto& s : sizes) {
    const int W = s[0], H = s[1];
    std::vector<uint8_t> img((size_t)W * H * 3);
    syn_image(1000u + W * 7u + H, W, H, 12, (W + H) & 1, 20.0, 5.0, img.data());
    std::vector<double> E;
    std::vector<uint8_t> keep;
    const int64_t ns = edge_all(img.data(), W, H, &E, &keep);
    CHECK(ns >= 0);
    int64_t kept = 0, ones = 0;
    for (size_t i = 0; i < E.size(); ++i) {
      kept += keep[i] != 0;
      ones += E[i] == 1.0;
      CHECK(std::isfinite(E[i]) && E[i] >= 0.0);
    }
    CHECK(kept == ns);
    CHECK(ns == 0 || ones >= 1);  // the median survivor maps to exactly 1
  }
  // views below 3x3 are rejected
  uint8_t tiny[2 * 5 * 3] = {0};
  std::vector<double> Et(10);
  CHECK(orc_edge_view(tiny, 5, 2, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                      Et.data(), nullptr, nullptr, nullptr) == -1);
  // a ramp R = G = B = x: gx = 2048000 from column 3, survivors only at column 3
  {
    const int W = 20, H = 12;
    std::vector<uint8_t> img((size_t)W * H * 3);
    for (int y = 0; y < H; ++y)
      for (int x = 0; x < W; ++x)
        for (int c = 0; c < 3; ++c) img[((size_t)y * W + x) * 3 + c] = (uint8_t)x;
    std::vector<uint8_t> keep;
    std::vector<int64_t> gx;
    CHECK(edge_all(img.data(), W, H, nullptr, &keep, &gx) == H);
    for (int y = 0; y < H; ++y) {
      CHECK(gx[(size_t)y * W + 5] == 2048000);
      for (int x = 0; x < W; ++x) CHECK((keep[(size_t)y * W + x] != 0) == (x == 3));
    }
  }
  // an ideal step: one survivor per row, at column k - 1, with map value 1
  {
    const int W = 20, H = 12, k = 10;
    std::vector<uint8_t> img((size_t)W * H * 3, 0);
    for (int y = 0; y < H; ++y)
      for (int x = k; x < W; ++x)
        for (int c = 0; c < 3; ++c) img[((size_t)y * W + x) * 3 + c] = 255;
    std::vector<double> E;
    std::vector<uint8_t> keep;
    CHECK(edge_all(img.data(), W, H, &E, &keep) == H);
    for (int y = 0; y < H; ++y) CHECK(keep[(size_t)y * W + k - 1] == 1 && E[(size_t)y * W + k - 1] == 1.0);
  }
  // suppression alone on a random gradient field
  {
    const int W = 11, H = 9;
    std::vector<int64_t> gx(W * H), gy(W * H), M(W * H);
    std::vector<uint8_t> bin(W * H), keep(W * H);
    std::vector<double> margin(W * H);
    uint64_t z = 12345;
    for (int i = 0; i < W * H; ++i) {
      z = z * 6364136223846793005ull + 1442695040888963407ull;
      gx[i] = (int64_t)(z >> 40) - (1 << 23);
      gy[i] = (int64_t)((z >> 16) & 0xFFFFFF) - (1 << 23);
    }
    orc_nms(gx.data(), gy.data(), W, H, M.data(), bin.data(), keep.data(), margin.data());
    for (int i = 0; i < W * H; ++i) CHECK(M[i] == gx[i] * gx[i] + gy[i] * gy[i] && margin[i] >= 0.0);
  }
  // a packed batch: full views and 2x downsamples, equal to the views alone
  {
    const int n = 3;
    const uint64_t seeds[n] = {7, 8, 9};
    const int32_t fw[n] = {64, 61, 33}, fh[n] = {48, 40, 9}, d2[n] = {0, 1, 0};
    int32_t W[n], H[n];
    int64_t in_off[n], out_off[n], ib = 0, ob = 0;
    for (int v = 0; v < n; ++v) {
      W[v] = d2[v] ? fw[v] / 2 : fw[v];
      H[v] = d2[v] ? fh[v] / 2 : fh[v];
      in_off[v] = ib;
      out_off[v] = ob;
      ib += (int64_t)W[v] * H[v] * 3 + 5;  // ragged gaps between views
      ob += (int64_t)W[v] * H[v] + 3;
    }
    std::vector<uint8_t> rgb(ib);
    syn_image_batch(n, seeds, fw, fh, d2, 10, 1, 20.0, 5.0, in_off, rgb.data());
    std::vector<double> E(ob), med(n);
    std::vector<uint8_t> keep(ob);
    std::vector<int64_t> ns(n);
    orc_edge_batch(rgb.data(), n, W, H, in_off, out_off, E.data(), keep.data(), med.data(), ns.data(), 1);
    for (int v = 0; v < n; ++v) {
      std::vector<double> Ev;
      CHECK(edge_all(rgb.data() + in_off[v], W[v], H[v], &Ev) == ns[v]);
      CHECK(std::memcmp(Ev.data(), E.data() + out_off[v], Ev.size() * sizeof(double)) == 0);
    }
    std::vector<uint8_t> d((size_t)W[1] * H[1] * 3);  // view 1 is the 2x downsample of a 61x40 render
    syn_image_down2(seeds[1], fw[1], fh[1], 10, 1, 20.0, 5.0, d.data());
    CHECK(std::memcmp(d.data(), rgb.data() + in_off[1], d.size()) == 0);
    int32_t vw[5], vh[5];
    syn_view_sizes(3, 5, 1000, 1560, 1.5, 1.7778, vw, vh);
    for (int v = 0; v < 5; ++v) CHECK(vw[v] >= 1000 && vw[v] <= 1560 && vh[v] > 500 && vh[v] < 1100);
  }
}

static void las_checks() {
  double R[9];
  const double qz[4] = {0, 0, 0, 0};
  orc_quat_to_R(qz, R);
  CHECK(R[0] == 1.0 && R[4] == 1.0 && R[8] == 1.0 && R[1] == 0.0);
  CHECK(std::fabs(orc_opacity(0.0, 0.6) - std::log(0.3 / 0.7)) < 1e-14);
  CHECK(std::isfinite(orc_opacity(-200.0, 0.6)) && std::isfinite(orc_opacity(200.0, 0.6)));
  for (int F : {0, 5}) {
    const int64_t N = 5000, K = 1000;
    for (int64_t cap : {N + K, N + K - 1}) {
      std::vector<float> means(cap * 3, 0.0f), ls(cap * 3, 0.0f), q(cap * 4, 0.0f), op(cap, 0.0f),
          feats(cap * (F > 0 ? F : 1), 0.5f);
      syn_gaussians(11, N, -4.0, 0.5, means.data(), ls.data(), q.data(), op.data());
      std::vector<uint8_t> mask(cap, 0);
      syn_mask(12, N, K, mask.data());
      std::vector<double> mo(cap * 3), lo(cap * 3), qo(cap * 4), oo(cap), fo(cap * (F > 0 ? F : 1));
      std::vector<int32_t> idx(cap), axis(cap);
      int64_t Ko = -1, cnt = -1;
      const int32_t st = orc_las(N, cap, means.data(), ls.data(), q.data(), op.data(), feats.data(), F, mask.data(),
                                 0.5, 0.85, 0.6, mo.data(), lo.data(), qo.data(), oo.data(), fo.data(), idx.data(),
                                 axis.data(), &Ko, &cnt);
      CHECK(Ko == K);
      if (cap == N + K) {
        CHECK(st == 0 && cnt == N + K);
        for (int64_t r = 0; r < K; ++r) {
          const int64_t i = idx[r], j = N + r;
          CHECK(r == 0 || idx[r] > idx[r - 1]);
          for (int k = 0; k < 3; ++k)  // the children's midpoint is the parent's mean
            CHECK(std::fabs(0.5 * (mo[i * 3 + k] + mo[j * 3 + k]) - means[i * 3 + k]) < 1e-12);
        }
      } else {
        CHECK(st == -6 && cnt == N);
      }
    }
  }
  // an empty selection and an empty set
  {
    float z[4] = {0, 0, 0, 0};
    uint8_t m[1] = {0};
    double d[4];
    int32_t i[1], a[1];
    int64_t Ko = -1, cnt = -1;
    CHECK(orc_las(0, 1, z, z, z, z, z, 0, m, 0.5, 0.85, 0.6, d, d, d, d, d, i, a, &Ko, &cnt) == 0 && Ko == 0 &&
          cnt == 0);
    CHECK(orc_las(1, 1, z, z, z, z, z, 0, m, 0.5, 0.85, 0.6, d, d, d, d, d, i, a, &Ko, &cnt) == 0 && Ko == 0 &&
          cnt == 1);
  }
}

static void contribution_checks() {
  const int32_t W[2] = {40, 3}, H[2] = {30, 5};
  for (int32_t order : {0, 1}) {
    const int64_t G = 300;
    std::vector<int64_t> off(G + 1, 0);
    const int64_t n = syn_contrib_count(21, G, 2, W, H, 3, off.data());
    CHECK(n > 0 && off[G] == n);
    std::vector<int32_t> g(n), v(n), p(n);
    std::vector<float> w(n);
    syn_contrib_fill(21, G, 2, W, H, 3, off.data(), order, g.data(), v.data(), p.data(), w.data());
    for (int64_t c = 0; c < n; ++c) {
      CHECK(g[c] >= 0 && g[c] < G && v[c] >= 0 && v[c] < 2);
      CHECK(p[c] >= 0 && p[c] < W[v[c]] * H[v[c]] && w[c] > 0.0f && w[c] <= 1.0f);
    }
  }
}

static void abi_checks() {
  using namespace igsp;
  uint8_t* img = reinterpret_cast<uint8_t*>(uintptr_t(0x7F0000000000));
  float* out = reinterpret_cast<float*>(uintptr_t(0x7F1000000000));
  igsp_view views[2] = {{16, 8, 0, 0}, {5, 3, 16 * 8 * 3, 16 * 8}};
  EdgeExtent ext{};
  CHECK(validate_edge(img, views, 2, out, nullptr, &ext) == IGSP_OK && ext.pixels == 16 * 8 + 15);
  CHECK(validate_edge(img, views, -1, out, nullptr, &ext) == IGSP_ERR_DIMS);
  CHECK(validate_edge(img + 1, views, 2, out, nullptr, &ext) == IGSP_ERR_ALIGN);
  CHECK(validate_edge(nullptr, views, 2, out, nullptr, &ext) == IGSP_ERR_NULL);
  igsp_view bad = {65536, 32768, 0, 0};
  CHECK(validate_edge(img, &bad, 1, out, nullptr, &ext) == IGSP_ERR_DIMS);
  igsp_edge_opts o{};
  o.precision = 7;
  CHECK(validate_edge(img, views, 2, out, &o, &ext) == IGSP_ERR_PARAM);
  o.precision = IGSP_BF16;
  o.wg_waves = 3;
  CHECK(validate_edge(img, views, 2, out, &o, &ext) == IGSP_ERR_PARAM);
  float* f = out;
  int64_t cnt_dummy = 0;
  igsp_gaussians g{f, f, f, f, nullptr, 0, &cnt_dummy, 100};
  int32_t i32 = 0;
  igsp_las_out lo{&i32, &i32, nullptr};
  igsp_las_params pr{0.5f, 0.85f, 0.6f};
  CHECK(validate_las(&g, img, &lo, &pr) == IGSP_OK);
  pr.alpha = NAN;
  CHECK(validate_las(&g, img, &lo, &pr) == IGSP_ERR_PARAM);
  g.capacity = -1;
  CHECK(validate_las(&g, img, &lo, nullptr) == IGSP_ERR_DIMS);
  g.capacity = 100;
  g.feat_dim = 4;
  CHECK(validate_las(&g, img, &lo, nullptr) == IGSP_ERR_NULL);
  CHECK(validate_las(nullptr, img, &lo, nullptr) == IGSP_ERR_NULL);
  int32_t ig[1] = {0};
  igsp_contributions c{ig, ig, ig, f, 5};
  igsp_select_params sp{0.0f, 0, 100};
  int64_t sc = 0;
  CHECK(validate_select(f, views, 2, &c, f, &cnt_dummy, 100, &sp, img, &sc) == IGSP_OK);
  sp.warmup = 2;
  CHECK(validate_select(f, views, 2, &c, f, &cnt_dummy, 100, &sp, img, &sc) == IGSP_ERR_PARAM);
  for (int32_t code = -12; code <= 1; ++code) CHECK(igsp_status_string(code) != nullptr);
  CHECK(std::fabs(igsp_lr_exponential(50, 0.02, 0.002, 100) - 0.02 * std::sqrt(0.1)) < 1e-15);
  CHECK(std::isnan(igsp_lr_exponential(5, 0.0, 0.002, 100)) && std::isnan(igsp_lr_exponential(5, 0.1, 0.2, 0)));
  CHECK(igsp_lr_exponential(-5, 0.02, 0.002, 100) == 0.02);
}

int main() {
  edge_checks();
  las_checks();
  contribution_checks();
  abi_checks();
  if (g_fail) {
    std::fprintf(stderr, "%d checks failed\n", g_fail);
    return 1;
  }
  std::printf("sanitized run: all checks passed\n");
  return 0;
}

// C ABI of the SLRF eigensolver: context, workspace carving, filter
// application (Algorithm 1's shifted solves and filter sum) and the outer
// subspace iteration with Rayleigh-Ritz and residuals.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/slrf.h"
#include "../../include/slrf_testing.h"
#include "dense.h"
#include "kernels.h"

using namespace slrf;

namespace {

constexpr int kRowsPerBlock = 8;
constexpr int kSubBand = 1024;  // rows per sub-band of the sparse-product row order

size_t al(size_t x) { return (x + 255) & ~size_t(255); }

struct Carver {
  char* base;
  size_t off = 0, cap = 0;
  template <typename T>
  T* take(size_t count) {
    T* p = reinterpret_cast<T*>(base + off);
    off = al(off + count * sizeof(T));
    return p;
  }
};

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Sizes of the per-call workspace regions for (n, L, N).
struct DynLayout {
  size_t krylov64 = 0, outer = 0, total = 0;
};

// ILU(0) runs one thread per column over all rows: only for narrow patterns.
bool ilu_allowed(int64_t n, int64_t nnz) { return nnz <= 5 * n; }

size_t krylov_bytes_fp64(int64_t n, int64_t nnz, int64_t L, int64_t N) {
  const int64_t K = N * L;
  const int64_t nrb = (n + kRowsPerBlock - 1) / kRowsPerBlock;
  size_t b = 0;
  b += 6 * al((size_t)n * K * 16);          // x r ph v sh t
  if (ilu_allowed(n, nnz)) b += 2 * al((size_t)n * K * 16) + al((size_t)N * nnz * 16);  // p s factors
  b += al((size_t)n * L * 8);               // rhat = B X
  b += 2 * al((size_t)n * N * 16);          // d, dinv
  b += al((size_t)N * 16) + al((size_t)K * 16) + al((size_t)2 * N * 8);  // sigma, sigma_col, w
  b += al((size_t)kMaxGrid * K * 16) + al((size_t)kMaxGrid * K * 8);      // partials [G][K]
  b += 4 * al((size_t)K * 16) + 2 * al((size_t)K * 8) + 2 * al((size_t)K * 4) + al(256);
  return b;
}

// MIXED: FP32 Krylov state (+ per-column complex shadow residual, p and s for
// ILU) and the FP64 accumulator Y, defect R and right-hand side F.
size_t krylov_bytes_mixed(int64_t n, int64_t nnz, int64_t L, int64_t N) {
  const int64_t K = N * L;
  size_t b = 0;
  b += 7 * al((size_t)n * K * 8);                                           // x r ph v sh t rhat (FP32)
  if (ilu_allowed(n, nnz)) b += 2 * al((size_t)n * K * 8) + al((size_t)N * nnz * 8);
  b += 2 * al((size_t)n * K * 16) + al((size_t)n * L * 8);                  // Y R (FP64), F
  b += 2 * al((size_t)n * N * 8);                                           // d, dinv (FP32)
  b += al((size_t)N * 8) + al((size_t)K * 8) + al((size_t)K * 16) + al((size_t)2 * N * 8);
  b += al((size_t)kMaxGrid * K * 8) + al((size_t)kMaxGrid * K * 4) + al((size_t)kMaxGrid * K * 8);
  b += 4 * al((size_t)K * 8) + 2 * al((size_t)K * 4) + 2 * al((size_t)K * 4) + 3 * al((size_t)K * 8) + al(256);
  return b;
}

size_t krylov_bytes(int64_t n, int64_t nnz, int64_t L, int64_t N, int precision) {
  return precision == SLRF_MIXED ? krylov_bytes_mixed(n, nnz, L, N) : krylov_bytes_fp64(n, nnz, L, N);
}

size_t outer_bytes(int64_t n, int64_t L) {
  const int nch = gram_chunks((int)n, (int)L);
  const int64_t nrr = (n + 255) / 256;
  size_t b = 0;
  b += 5 * al((size_t)n * L * 8);                   // V U WA WB X
  b += al((size_t)nch * 2 * L * L * 8);             // gram partials
  b += 3 * al((size_t)L * L * 8);                   // GA GB Z
  b += al((size_t)L * 8);                           // theta
  b += al((size_t)(nrr * 2 * L + 2 * L) * 8);       // residual partials
  return b;
}

}  // namespace

struct slrf_ctx_s {
  int64_t n = 0, nnz = 0;
  hipStream_t stream = nullptr;
  slrf_options opt{};
  char* ws = nullptr;
  size_t ws_bytes = 0;
  size_t static_bytes = 0;
  int64_t max_L = 0;
  int32_t max_N = 0;
  int* rowptr = nullptr;
  int* col = nullptr;
  ab_pair<double>* ab64 = nullptr;
  double* diagA = nullptr;
  double* diagB = nullptr;
  ab_pair<float>* ab32 = nullptr;  // FP32 copies for the mixed path
  float* diagA32 = nullptr;
  float* diagB32 = nullptr;
  std::string err;
  bool verbose = false;
  bool use_ilu = false;
  int* diagpos = nullptr;
  int* sched = nullptr;     // sparse-product row order, null = natural order
  // host copy of the merged CSR, kept for the per-pole ILU(0) factorisations
  std::vector<int32_t> h_rp, h_cl, h_dpos;
  std::vector<double> h_ab;
  LaunchTimer timer;
  std::vector<hipEvent_t> events;
  ~slrf_ctx_s() {
    for (hipEvent_t e : events)
      if (e) (void)hipEventDestroy(e);
  }
};

namespace {

slrf_status fail(slrf_ctx ctx, slrf_status s, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return s;
}

#define HIPCHK(ctx, call)                                                                  \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(ctx, SLRF_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr int kTimerSlots = 512;

size_t static_bytes_for(int64_t n, int64_t nnz) {
  return al((size_t)(n + 1) * 4) + al((size_t)nnz * 4) + al((size_t)nnz * 16) + 2 * al((size_t)n * 8) +
         al((size_t)n * 4) + al(kTimerSlots * 4) + al((size_t)n * 4) + al((size_t)nnz * 8) + 2 * al((size_t)n * 4);
}

// Row order of the sparse products.  With upper bandwidth H (max j - i), the
// neighbours of row i lie in [i - H, i + H].  Rows are cut into chunks of H and
// each chunk into S sub-bands of about kSubBand rows; the order visits sub-band
// s of chunk 0, 1, 2, ... before sub-band s + 1, so consecutive rows in the
// order have overlapping neighbourhoods (for a lexicographic 3D grid: a narrow
// (x, y) band marching along z).  Returns false (natural order) when H is small.
bool band_schedule(int64_t n, const std::vector<int32_t>& rp, const std::vector<int32_t>& cl,
                   std::vector<int32_t>& order) {
  int64_t H = 0;
  for (int64_t i = 0; i < n; ++i)
    if (rp[i + 1] > rp[i]) H = std::max<int64_t>(H, (int64_t)cl[rp[i + 1] - 1] - i);
  if (H <= 2 * kSubBand || H >= n) return false;
  const int64_t S = (H + kSubBand - 1) / kSubBand, band = (H + S - 1) / S, nchunk = (n + H - 1) / H;
  order.clear();
  order.reserve(n);
  for (int64_t sb = 0; sb < S; ++sb)
    for (int64_t k = 0; k < nchunk; ++k) {
      const int64_t a = k * H + sb * band, b = std::min({k * H + (sb + 1) * band, (k + 1) * H, n});
      for (int64_t r = a; r < b; ++r) order.push_back((int32_t)r);
    }
  return (int64_t)order.size() == n;
}

double merged_csr_bytes(const slrf_ctx ctx, size_t value_bytes) {
  return (double)(ctx->n + 1) * 4 + (double)ctx->nnz * (4 + value_bytes);
}

// Reads back the event pairs and tile counters of the current window into the
// kernel statistics, then clears the window.
slrf_status harvest_timer(slrf_ctx ctx, int64_t total_tiles, slrf_filter_stats* fs) {
  LaunchTimer& tm = ctx->timer;
  if (tm.used == 0) return SLRF_OK;
  std::vector<int> cnt(tm.used);
  HIPCHK(ctx, hipMemcpyAsync(cnt.data(), tm.d_counts, 4 * (size_t)tm.used, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  for (int u = 0; u < tm.used; ++u) {
    float ms = 0;
    HIPCHK(ctx, hipEventElapsedTime(&ms, tm.events[2 * u], tm.events[2 * u + 1]));
    const LaunchTimer::Rec& r = tm.recs[u];
    const double bytes = r.tile_bytes * (double)cnt[u] / (double)total_tiles + (cnt[u] > 0 ? r.fixed : 0.0);
    if (r.kind == 0) {
      fs->spmm_seconds += 1e-3 * ms;
      fs->spmm_launches += 1;
      fs->spmm_bytes += bytes;
    } else {
      fs->update_seconds += 1e-3 * ms;
      fs->update_launches += 1;
      fs->update_bytes += bytes;
    }
  }
  tm.used = 0;
  launch_fill_zero(ctx->stream, tm.d_counts, 4 * (size_t)tm.capacity);
  return SLRF_OK;
}

// ILU(0) of A - sigma B on the merged pattern (row-wise IKJ elimination without
// fill); the U diagonal is returned inverted.
bool ilu0_factor(const slrf_ctx ctx, std::complex<double> sigma, std::vector<std::complex<double>>& f) {
  const int64_t n = ctx->n, nnz = ctx->nnz;
  const auto& rp = ctx->h_rp;
  const auto& cl = ctx->h_cl;
  const auto& dp = ctx->h_dpos;
  f.resize(nnz);
  for (int64_t k = 0; k < nnz; ++k) f[k] = std::complex<double>(ctx->h_ab[2 * k], 0.0) - sigma * ctx->h_ab[2 * k + 1];
  for (int64_t i = 0; i < n; ++i) {
    for (int32_t k = rp[i]; k < dp[i]; ++k) {
      const int32_t c = cl[k];
      f[k] /= f[dp[c]];
      const std::complex<double> lik = f[k];
      int32_t a = k + 1, b = dp[c] + 1;
      while (a < rp[i + 1] && b < rp[c + 1]) {
        if (cl[a] == cl[b]) {
          f[a] -= lik * f[b];
          ++a;
          ++b;
        } else if (cl[a] < cl[b]) {
          ++a;
        } else {
          ++b;
        }
      }
    }
    if (std::abs(f[dp[i]]) == 0.0 || !std::isfinite(std::abs(f[dp[i]]))) return false;
  }
  for (int64_t i = 0; i < n; ++i) f[dp[i]] = 1.0 / f[dp[i]];
  return true;
}

std::mutex g_design_mu;
std::map<std::tuple<int, double, double>, std::vector<double>> g_design_cache;

bool design_unit_cached(int N, double alpha, double beta, std::vector<double>& out /* 3N */) {
  std::lock_guard<std::mutex> lk(g_design_mu);
  auto key = std::make_tuple(N, alpha, beta);
  auto it = g_design_cache.find(key);
  if (it != g_design_cache.end()) {
    out = it->second;
    return true;
  }
  std::vector<double> xi(N), om(2 * N);
  if (!design_poles_unit(N, alpha, beta, xi.data(), om.data())) return false;
  out.assign(3 * N, 0.0);
  for (int j = 0; j < N; ++j) {
    out[j] = xi[j];
    out[N + 2 * j] = om[2 * j];
    out[N + 2 * j + 1] = om[2 * j + 1];
  }
  g_design_cache[key] = out;
  return true;
}

slrf_status check_poles(slrf_ctx ctx, const slrf_poles* p) {
  if (!p || p->n_poles < 1 || !p->sigma || !p->weight)
    return fail(ctx, SLRF_E_INVALID_ARG, "pole set is NULL or empty");
  if (p->n_poles > ctx->max_N) return fail(ctx, SLRF_E_INVALID_ARG, "more poles than the workspace was sized for");
  for (int j = 0; j < p->n_poles; ++j) {
    const double a = p->sigma[2 * j], b = p->sigma[2 * j + 1], c = p->weight[2 * j], d = p->weight[2 * j + 1];
    if (!std::isfinite(a) || !std::isfinite(b) || !std::isfinite(c) || !std::isfinite(d))
      return fail(ctx, SLRF_E_INVALID_ARG, "non-finite pole or weight");
    if (!(b > 0)) return fail(ctx, SLRF_E_INVALID_ARG, "poles must lie in the upper half plane (Im sigma > 0)");
  }
  return SLRF_OK;
}

// Filter application into U (FP64 path).  Workspace carved from `cv`.
slrf_status filter_fp64(slrf_ctx ctx, Carver& cv, const slrf_poles* poles, int L, const double* X, double* U,
                        slrf_filter_stats* stats) {
  const double t0 = now_s();
  hipStream_t s = ctx->stream;
  const int n = (int)ctx->n, N = poles->n_poles;
  KGeom g = make_geom(n, N, L, kRowsPerBlock);
  g.sched = ctx->sched;
  const int K = g.K;
  KrylovState<double> st{};
  st.x = cv.take<cx<double>>((size_t)n * K);
  st.r = cv.take<cx<double>>((size_t)n * K);
  st.ph = cv.take<cx<double>>((size_t)n * K);
  st.v = cv.take<cx<double>>((size_t)n * K);
  st.sh = cv.take<cx<double>>((size_t)n * K);
  st.t = cv.take<cx<double>>((size_t)n * K);
  cx<double>* fac = nullptr;
  if (ctx->use_ilu) {
    st.p = cv.take<cx<double>>((size_t)n * K);
    st.s = cv.take<cx<double>>((size_t)n * K);
    fac = cv.take<cx<double>>((size_t)N * ctx->nnz);
  }
  double* rhat = cv.take<double>((size_t)n * L);
  cx<double>* d = cv.take<cx<double>>((size_t)n * N);
  cx<double>* dinv = cv.take<cx<double>>((size_t)n * N);
  cx<double>* sig = cv.take<cx<double>>(N);
  cx<double>* sigc = cv.take<cx<double>>(K);
  double* w = cv.take<double>(2 * N);
  st.part_a = cv.take<cx<double>>((size_t)g.G * K);
  st.part_b = cv.take<double>((size_t)g.G * K);
  st.rho = cv.take<cx<double>>(K);
  st.alpha = cv.take<cx<double>>(K);
  st.omega = cv.take<cx<double>>(K);
  st.beta = cv.take<cx<double>>(K);
  st.fnorm = cv.take<double>(K);
  st.rnorm = cv.take<double>(K);
  st.flags = cv.take<int>(K);
  st.iters = cv.take<int>(K);
  int* d_count = cv.take<int>(64);
  if (cv.off > cv.cap) return fail(ctx, SLRF_E_WORKSPACE, "workspace too small for this L and pole count");
  st.rhat = rhat;
  st.d = d;
  st.dinv = dinv;
  st.sigma_col = sigc;

  std::vector<double> hsig(2 * N), hsigc(2 * (size_t)K);
  for (int j = 0; j < N; ++j) {
    hsig[2 * j] = poles->sigma[2 * j];
    hsig[2 * j + 1] = poles->sigma[2 * j + 1];
    for (int l = 0; l < L; ++l) {
      hsigc[2 * ((size_t)j * L + l)] = poles->sigma[2 * j];
      hsigc[2 * ((size_t)j * L + l) + 1] = poles->sigma[2 * j + 1];
    }
  }
  HIPCHK(ctx, hipMemcpyAsync(sig, hsig.data(), 16 * N, hipMemcpyHostToDevice, s));
  HIPCHK(ctx, hipMemcpyAsync(sigc, hsigc.data(), 16 * (size_t)K, hipMemcpyHostToDevice, s));
  HIPCHK(ctx, hipMemcpyAsync(w, poles->weight, 16 * N, hipMemcpyHostToDevice, s));

  IluFactors<double> ilu{};
  std::vector<std::complex<double>> hf;
  if (ctx->use_ilu) {
    hf.resize((size_t)N * ctx->nnz);
    std::vector<std::complex<double>> fj;
    for (int j = 0; j < N; ++j) {
      if (!ilu0_factor(ctx, {poles->sigma[2 * j], poles->sigma[2 * j + 1]}, fj))
        return fail(ctx, SLRF_E_BREAKDOWN, "zero pivot in the ILU(0) factorisation of the shifted operator");
      std::copy(fj.begin(), fj.end(), hf.begin() + (size_t)j * ctx->nnz);
    }
    HIPCHK(ctx, hipMemcpyAsync(fac, hf.data(), 16 * hf.size(), hipMemcpyHostToDevice, s));
    ilu = {ctx->rowptr, ctx->col, ctx->diagpos, fac, ctx->nnz};
  }
  launch_jacobi_diag<double>(s, n, N, ctx->diagA, ctx->diagB, sig, d, dinv);
  launch_spmm_real<double>(s, n, L, ctx->rowptr, ctx->col, ctx->ab64, X, nullptr, rhat);
  launch_init<double>(s, g, st, rhat);
  launch_init_scalars<double>(s, g, st);
  HIPCHK(ctx, hipGetLastError());

  const int maxit = std::max(1, ctx->opt.inner_maxit);
  const int every = std::max(1, std::min(ctx->opt.check_every, 64));
  const double tol = ctx->opt.inner_tol;
  LaunchTimer* tm = ctx->opt.profile ? &ctx->timer : nullptr;
  const double mbytes = merged_csr_bytes(ctx, 16);
  slrf_filter_stats ks{};
  int it = 0;
  while (it < maxit) {
    const int chunk = std::min(every, maxit - it);
    for (int q = 0; q < chunk; ++q, ++it)
      launch_iteration<double>(s, g, st, ctx->rowptr, ctx->col, ctx->ab64, tol, maxit, it == 0,
                               ctx->use_ilu ? &ilu : nullptr, tm, mbytes);
    launch_count_active(s, K, st.flags, d_count);
    HIPCHK(ctx, hipGetLastError());
    int active = 0;
    HIPCHK(ctx, hipMemcpyAsync(&active, d_count, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    if (tm) {
      slrf_status hs = harvest_timer(ctx, (int64_t)g.G * g.nct, &ks);
      if (hs != SLRF_OK) return hs;
    }
    if (active == 0) break;
  }
  launch_filter_sum<double>(s, n, L, N, st.x, w, U, false);
  HIPCHK(ctx, hipGetLastError());

  if (stats) {
    std::vector<int> fl(K), its(K);
    std::vector<double> rn(K), fn(K);
    HIPCHK(ctx, hipMemcpyAsync(fl.data(), st.flags, 4 * (size_t)K, hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipMemcpyAsync(its.data(), st.iters, 4 * (size_t)K, hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipMemcpyAsync(rn.data(), st.rnorm, 8 * (size_t)K, hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipMemcpyAsync(fn.data(), st.fnorm, 8 * (size_t)K, hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    slrf_filter_stats fs{};
    double sum_it = 0;
    for (int c = 0; c < K; ++c) {
      fs.max_iterations = std::max(fs.max_iterations, its[c]);
      sum_it += its[c];
      fs.spmv += 2 * (int64_t)its[c] - (fl[c] == COL_HALF_CONVERGED ? 1 : 0);
      if (fl[c] == COL_BREAKDOWN) fs.n_breakdown++;
      if (fl[c] == COL_MAXIT) fs.n_maxit++;
      const double rr = fn[c] > 0 ? rn[c] / fn[c] : 0.0;
      fs.max_relres = std::max(fs.max_relres, rr);
    }
    fs.mean_iterations = K ? sum_it / K : 0.0;
    HIPCHK(ctx, hipStreamSynchronize(s));
    fs.seconds = now_s() - t0;
    fs.spmm_seconds = ks.spmm_seconds;
    fs.spmm_launches = ks.spmm_launches;
    fs.spmm_bytes = ks.spmm_bytes;
    fs.update_seconds = ks.update_seconds;
    fs.update_launches = ks.update_launches;
    fs.update_bytes = ks.update_bytes;
    *stats = fs;
  }
  return SLRF_OK;
}

// Filter application with complex FP32 inner solves and FP64 defect correction:
// Y = 0; repeat { R = F - S Y (FP64); stop columns with ||R|| <= target ||F||;
// solve S D = R / ||R|| in FP32 (BiCGStab, relative tolerance inner_tol32);
// Y += ||R|| D } ; U = sum_j 2 Re(w_j Y_j).
constexpr double kInnerTol32 = 1e-6;
constexpr int kMaxRounds = 6;

slrf_status filter_mixed(slrf_ctx ctx, Carver& cv, const slrf_poles* poles, int L, const double* X, double* U,
                         slrf_filter_stats* stats, double target) {
  const double t0 = now_s();
  hipStream_t s = ctx->stream;
  const int n = (int)ctx->n, N = poles->n_poles;
  KGeom g = make_geom(n, N, L, kRowsPerBlock);
  g.sched = ctx->sched;
  const int K = g.K;
  KrylovState<float> st{};
  st.x = cv.take<cx<float>>((size_t)n * K);
  st.r = cv.take<cx<float>>((size_t)n * K);
  st.ph = cv.take<cx<float>>((size_t)n * K);
  st.v = cv.take<cx<float>>((size_t)n * K);
  st.sh = cv.take<cx<float>>((size_t)n * K);
  st.t = cv.take<cx<float>>((size_t)n * K);
  cx<float>* rhat = cv.take<cx<float>>((size_t)n * K);
  cx<float>* fac = nullptr;
  if (ctx->use_ilu) {
    st.p = cv.take<cx<float>>((size_t)n * K);
    st.s = cv.take<cx<float>>((size_t)n * K);
    fac = cv.take<cx<float>>((size_t)N * ctx->nnz);
  }
  cx<double>* Y = cv.take<cx<double>>((size_t)n * K);
  cx<double>* Rd = cv.take<cx<double>>((size_t)n * K);
  double* F = cv.take<double>((size_t)n * L);
  cx<float>* d = cv.take<cx<float>>((size_t)n * N);
  cx<float>* dinv = cv.take<cx<float>>((size_t)n * N);
  cx<float>* sig = cv.take<cx<float>>(N);
  cx<float>* sigc = cv.take<cx<float>>(K);
  cx<double>* sigc64 = cv.take<cx<double>>(K);
  double* w = cv.take<double>(2 * N);
  st.part_a = cv.take<cx<float>>((size_t)g.G * K);
  st.part_b = cv.take<float>((size_t)g.G * K);
  double* part64 = cv.take<double>((size_t)g.G * K);
  st.rho = cv.take<cx<float>>(K);
  st.alpha = cv.take<cx<float>>(K);
  st.omega = cv.take<cx<float>>(K);
  st.beta = cv.take<cx<float>>(K);
  st.fnorm = cv.take<float>(K);
  st.rnorm = cv.take<float>(K);
  st.flags = cv.take<int>(K);
  st.iters = cv.take<int>(K);
  double* fnorm64 = cv.take<double>(K);
  double* scale = cv.take<double>(K);
  double* relres = cv.take<double>(K);
  int* d_count = cv.take<int>(64);
  if (cv.off > cv.cap) return fail(ctx, SLRF_E_WORKSPACE, "workspace too small for this L and pole count");
  st.rhat = nullptr;
  st.rhat_cx = rhat;
  st.d = d;
  st.dinv = dinv;
  st.sigma_col = sigc;

  std::vector<float> hsig(2 * N), hsigc(2 * (size_t)K);
  std::vector<double> hsigc64(2 * (size_t)K);
  for (int j = 0; j < N; ++j) {
    hsig[2 * j] = (float)poles->sigma[2 * j];
    hsig[2 * j + 1] = (float)poles->sigma[2 * j + 1];
    for (int l = 0; l < L; ++l) {
      const size_t c = (size_t)j * L + l;
      hsigc[2 * c] = (float)poles->sigma[2 * j];
      hsigc[2 * c + 1] = (float)poles->sigma[2 * j + 1];
      hsigc64[2 * c] = poles->sigma[2 * j];
      hsigc64[2 * c + 1] = poles->sigma[2 * j + 1];
    }
  }
  HIPCHK(ctx, hipMemcpyAsync(sig, hsig.data(), 8 * N, hipMemcpyHostToDevice, s));
  HIPCHK(ctx, hipMemcpyAsync(sigc, hsigc.data(), 8 * (size_t)K, hipMemcpyHostToDevice, s));
  HIPCHK(ctx, hipMemcpyAsync(sigc64, hsigc64.data(), 16 * (size_t)K, hipMemcpyHostToDevice, s));
  HIPCHK(ctx, hipMemcpyAsync(w, poles->weight, 16 * N, hipMemcpyHostToDevice, s));
  IluFactors<float> ilu{};
  std::vector<cx<float>> hf;
  if (ctx->use_ilu) {
    hf.resize((size_t)N * ctx->nnz);
    std::vector<std::complex<double>> fj;
    for (int j = 0; j < N; ++j) {
      if (!ilu0_factor(ctx, {poles->sigma[2 * j], poles->sigma[2 * j + 1]}, fj))
        return fail(ctx, SLRF_E_BREAKDOWN, "zero pivot in the ILU(0) factorisation of the shifted operator");
      for (int64_t k = 0; k < ctx->nnz; ++k)
        hf[(size_t)j * ctx->nnz + k] = {(float)fj[k].real(), (float)fj[k].imag()};
    }
    HIPCHK(ctx, hipMemcpyAsync(fac, hf.data(), 8 * hf.size(), hipMemcpyHostToDevice, s));
    ilu = {ctx->rowptr, ctx->col, ctx->diagpos, fac, ctx->nnz};
  }
  launch_jacobi_diag<float>(s, n, N, ctx->diagA32, ctx->diagB32, sig, d, dinv);
  launch_spmm_real<double>(s, n, L, ctx->rowptr, ctx->col, ctx->ab64, X, nullptr, F);
  HIPCHK(ctx, hipGetLastError());

  const int maxit = std::max(1, ctx->opt.inner_maxit);
  const int every = std::max(1, std::min(ctx->opt.check_every, 64));
  LaunchTimer* tm = ctx->opt.profile ? &ctx->timer : nullptr;
  const double mbytes = merged_csr_bytes(ctx, 8);
  slrf_filter_stats fs{};
  double sum_it = 0;
  int rounds = 0;
  for (int round = 0; round <= kMaxRounds; ++round) {
    // defect and the columns still above the target
    launch_defect(s, g, ctx->rowptr, ctx->col, ctx->ab64, sigc64, F, round ? Y : nullptr, Rd, part64);
    launch_defect_norms(s, g, part64, target, round == 0, fnorm64, scale, relres, d_count);
    HIPCHK(ctx, hipGetLastError());
    int open = 0;
    HIPCHK(ctx, hipMemcpyAsync(&open, d_count, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    if (round > 0) fs.spmv += (int64_t)K;  // one product with S per column for the defect
    if (open == 0 || round == kMaxRounds) break;
    ++rounds;
    launch_mixed_rhs(s, g, round ? Rd : nullptr, F, scale, st, rhat);
    launch_init_scalars<float>(s, g, st);
    int it = 0;
    while (it < maxit) {
      const int chunk = std::min(every, maxit - it);
      for (int q = 0; q < chunk; ++q, ++it)
        launch_iteration<float>(s, g, st, ctx->rowptr, ctx->col, ctx->ab32, (float)kInnerTol32, maxit, it == 0,
                                ctx->use_ilu ? &ilu : nullptr, tm, mbytes);
      launch_count_active(s, K, st.flags, d_count);
      HIPCHK(ctx, hipGetLastError());
      int active = 0;
      HIPCHK(ctx, hipMemcpyAsync(&active, d_count, sizeof(int), hipMemcpyDeviceToHost, s));
      HIPCHK(ctx, hipStreamSynchronize(s));
      if (tm) {
        slrf_status hs = harvest_timer(ctx, (int64_t)g.G * g.nct, &fs);
        if (hs != SLRF_OK) return hs;
      }
      if (active == 0) break;
    }
    launch_accumulate(s, g, st.x, scale, Y, round == 0);
    std::vector<int> fl(K), its(K);
    HIPCHK(ctx, hipMemcpyAsync(fl.data(), st.flags, 4 * (size_t)K, hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipMemcpyAsync(its.data(), st.iters, 4 * (size_t)K, hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    for (int c = 0; c < K; ++c) {
      fs.max_iterations = std::max(fs.max_iterations, its[c]);
      sum_it += its[c];
      fs.spmv += 2 * (int64_t)its[c] - (fl[c] == COL_HALF_CONVERGED ? 1 : 0);
      if (fl[c] == COL_BREAKDOWN) fs.n_breakdown++;
      if (fl[c] == COL_MAXIT) fs.n_maxit++;
    }
  }
  launch_filter_sum<double>(s, n, L, N, Y, w, U, false);
  HIPCHK(ctx, hipGetLastError());
  std::vector<double> rr(K);
  HIPCHK(ctx, hipMemcpyAsync(rr.data(), relres, 8 * (size_t)K, hipMemcpyDeviceToHost, s));
  HIPCHK(ctx, hipStreamSynchronize(s));
  if (stats) {
    for (int c = 0; c < K; ++c) fs.max_relres = std::max(fs.max_relres, rr[c]);
    fs.mean_iterations = K ? sum_it / K : 0.0;
    fs.refinements = rounds;
    fs.seconds = now_s() - t0;
    *stats = fs;
  }
  return SLRF_OK;
}

// One Rayleigh-Ritz pass: Y = Xin Z with (Y^T A Y, Y^T B Y) = (diag(theta), I).
slrf_status rr_pass(slrf_ctx ctx, int L, const double* Xin, double* Y, double* WA, double* WB, double* part,
                    int nch, double* GA, double* GB, double* Zd, std::vector<double>& theta) {
  hipStream_t s = ctx->stream;
  const int n = (int)ctx->n;
  launch_spmm_real<double>(s, n, L, ctx->rowptr, ctx->col, ctx->ab64, Xin, WA, WB);
  launch_gram(s, n, L, Xin, WA, WB, part, nch, GA, GB);
  HIPCHK(ctx, hipGetLastError());
  std::vector<double> hA((size_t)L * L), hB((size_t)L * L), Z((size_t)L * L);
  HIPCHK(ctx, hipMemcpyAsync(hA.data(), GA, 8 * hA.size(), hipMemcpyDeviceToHost, s));
  HIPCHK(ctx, hipMemcpyAsync(hB.data(), GB, 8 * hB.size(), hipMemcpyDeviceToHost, s));
  HIPCHK(ctx, hipStreamSynchronize(s));
  theta.assign(L, 0.0);
  if (!projected_pencil(L, hA.data(), hB.data(), theta.data(), Z.data()))
    return fail(ctx, SLRF_E_BREAKDOWN, "projected pencil not solvable (non-finite or zero Gram matrix)");
  HIPCHK(ctx, hipMemcpyAsync(Zd, Z.data(), 8 * Z.size(), hipMemcpyHostToDevice, s));
  const double* xs[1] = {Xin};
  double* ys[1] = {Y};
  launch_gemm_nz(s, n, L, L, 1, xs, Zd, ys);
  HIPCHK(ctx, hipGetLastError());
  HIPCHK(ctx, hipStreamSynchronize(s));  // Z host buffer lifetime
  return SLRF_OK;
}

}  // namespace

extern "C" {

void slrf_default_options(slrf_options* o) {
  if (!o) return;
  o->precision = SLRF_FP64;
  o->inner_tol = 1e-10;
  o->inner_maxit = 1000;
  o->outer_tol = 1e-8;
  o->outer_maxit = 40;
  o->check_every = 10;
  o->seed = 1;
  o->precond = 0;
}

const char* slrf_status_string(slrf_status s) {
  switch (s) {
    case SLRF_OK: return "ok";
    case SLRF_E_INVALID_ARG: return "invalid argument";
    case SLRF_E_NOT_SPD: return "A or B has a non-positive or missing diagonal entry";
    case SLRF_E_WORKSPACE: return "workspace too small or misaligned";
    case SLRF_E_DEVICE: return "HIP runtime error";
    case SLRF_E_NOT_CONVERGED: return "outer iteration did not converge";
    case SLRF_E_SUBSPACE_TOO_SMALL: return "subspace too small: every Ritz value lies in the interval";
    case SLRF_E_BREAKDOWN: return "breakdown of the projected problem";
  }
  return "unknown status";
}

const char* slrf_last_error(slrf_ctx ctx) { return ctx ? ctx->err.c_str() : "null context"; }

slrf_status slrf_design_poles(int32_t N, double alpha, double beta, double gamma, double* sigma_out,
                              double* weight_out, double* sep_out) {
  if (N < 1 || N > 16 || !(alpha > 0) || !(beta > 0) || !(gamma > 0) || !sigma_out || !weight_out)
    return SLRF_E_INVALID_ARG;
  std::vector<double> u;
  if (!design_unit_cached(N, alpha, beta, u)) return SLRF_E_INVALID_ARG;
  std::complex<double> dphi = 0;
  for (int j = 0; j < N; ++j) {
    const std::complex<double> sg(gamma * u[j], gamma * u[j] * alpha);
    const std::complex<double> wj(gamma * u[N + 2 * j], gamma * u[N + 2 * j + 1]);
    sigma_out[2 * j] = sg.real();
    sigma_out[2 * j + 1] = sg.imag();
    weight_out[2 * j] = wj.real();
    weight_out[2 * j + 1] = wj.imag();
    dphi += -2.0 * (wj / ((gamma - sg) * (gamma - sg))).real();
  }
  if (sep_out) *sep_out = std::abs(dphi.real());
  return SLRF_OK;
}

slrf_status slrf_workspace_bytes(int64_t n, int64_t nnz, int64_t L, int32_t N, int32_t precision, size_t* bytes) {
  if (n < 1 || nnz < n || L < 1 || N < 1 || !bytes || n > INT32_MAX || nnz > INT32_MAX) return SLRF_E_INVALID_ARG;
  if (precision != SLRF_FP64 && precision != SLRF_MIXED) return SLRF_E_INVALID_ARG;
  *bytes = static_bytes_for(n, nnz) + krylov_bytes(n, nnz, L, N, precision) + outer_bytes(n, L);
  return SLRF_OK;
}

slrf_status slrf_create(slrf_ctx* out, int64_t n, const int32_t* a_rowptr, const int32_t* a_col,
                        const double* a_val, const int32_t* b_rowptr, const int32_t* b_col, const double* b_val,
                        void* d_workspace, size_t ws_bytes, int64_t max_L, int32_t max_N, const slrf_options* opt,
                        void* hip_stream) {
  if (!out) return SLRF_E_INVALID_ARG;
  *out = nullptr;
  slrf_ctx ctx = new (std::nothrow) slrf_ctx_s();
  if (!ctx) return SLRF_E_INVALID_ARG;
  auto bail = [&](slrf_status s, const std::string& m) {
    ctx->err = m;
    *out = ctx;  // keep the context so the caller can read the message
    return s;
  };
  if (n < 1 || n > INT32_MAX || !a_rowptr || !a_col || !a_val || !b_rowptr || !b_col || !b_val || max_L < 1 ||
      max_N < 1)
    return bail(SLRF_E_INVALID_ARG, "bad size or NULL argument");
  if (opt) ctx->opt = *opt; else slrf_default_options(&ctx->opt);
  if (ctx->opt.precision != SLRF_FP64 && ctx->opt.precision != SLRF_MIXED)
    return bail(SLRF_E_INVALID_ARG, "unknown precision");
  ctx->n = n;
  ctx->verbose = getenv("SLRF_VERBOSE") != nullptr;
  ctx->stream = (hipStream_t)hip_stream;
  ctx->max_L = max_L;
  ctx->max_N = max_N;
  // validate and merge the two patterns
  auto check_csr = [&](const int32_t* rp, const int32_t* cl, const double* v, const char* name) -> std::string {
    if (rp[0] != 0) return std::string(name) + ": row_ptr[0] != 0";
    for (int64_t i = 0; i < n; ++i) {
      if (rp[i + 1] < rp[i]) return std::string(name) + ": row_ptr not non-decreasing";
      for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
        if (cl[k] < 0 || cl[k] >= n) return std::string(name) + ": column index out of range";
        if (k > rp[i] && cl[k] <= cl[k - 1]) return std::string(name) + ": columns not strictly increasing";
        if (!std::isfinite(v[k])) return std::string(name) + ": non-finite value";
      }
    }
    return "";
  };
  std::string m1 = check_csr(a_rowptr, a_col, a_val, "A");
  if (!m1.empty()) return bail(SLRF_E_INVALID_ARG, m1);
  std::string m2 = check_csr(b_rowptr, b_col, b_val, "B");
  if (!m2.empty()) return bail(SLRF_E_INVALID_ARG, m2);
  std::vector<int32_t> rp(n + 1, 0), cl, dpos(n, -1);
  std::vector<double> ab, dA(n, 0.0), dB(n, 0.0);
  cl.reserve(std::max(a_rowptr[n], b_rowptr[n]));
  ab.reserve(2 * (size_t)std::max(a_rowptr[n], b_rowptr[n]));
  for (int64_t i = 0; i < n; ++i) {
    int32_t ka = a_rowptr[i], kb = b_rowptr[i];
    const int32_t ea = a_rowptr[i + 1], eb = b_rowptr[i + 1];
    while (ka < ea || kb < eb) {
      const int32_t ca = ka < ea ? a_col[ka] : INT32_MAX, cb = kb < eb ? b_col[kb] : INT32_MAX;
      const int32_t c = std::min(ca, cb);
      const double va = (ca == c) ? a_val[ka++] : 0.0;
      const double vb = (cb == c) ? b_val[kb++] : 0.0;
      cl.push_back(c);
      ab.push_back(va);
      ab.push_back(vb);
      if (c == i) {
        dA[i] = va;
        dB[i] = vb;
        dpos[i] = (int32_t)cl.size() - 1;
      }
    }
    rp[i + 1] = (int32_t)cl.size();
  }
  for (int64_t i = 0; i < n; ++i)
    if (!(dA[i] > 0) || !(dB[i] > 0))
      return bail(SLRF_E_NOT_SPD, "row " + std::to_string(i) + ": diagonal of A or B not positive");
  const int64_t nnz = (int64_t)cl.size();
  ctx->nnz = nnz;
  if (ctx->opt.precond < 0 || ctx->opt.precond > 2) return bail(SLRF_E_INVALID_ARG, "unknown preconditioner");
  if (ctx->opt.precond == 2 && !ilu_allowed(n, nnz))
    return bail(SLRF_E_INVALID_ARG, "ILU(0) needs a narrow pattern (nnz <= 5 n)");
  ctx->use_ilu = ctx->opt.precond == 2 || (ctx->opt.precond == 0 && ilu_allowed(n, nnz));
  if (((uintptr_t)d_workspace & 255) != 0 || !d_workspace) return bail(SLRF_E_WORKSPACE, "workspace not 256-byte aligned");
  size_t need = 0;
  if (slrf_workspace_bytes(n, nnz, max_L, max_N, ctx->opt.precision, &need) != SLRF_OK)
    return bail(SLRF_E_INVALID_ARG, "bad sizes");
  if (ws_bytes < need)
    return bail(SLRF_E_WORKSPACE, "workspace has " + std::to_string(ws_bytes) + " bytes, needs " + std::to_string(need));
  ctx->ws = (char*)d_workspace;
  ctx->ws_bytes = ws_bytes;
  Carver cv{ctx->ws, 0, ws_bytes};
  ctx->rowptr = cv.take<int>(n + 1);
  ctx->col = cv.take<int>(nnz);
  ctx->ab64 = cv.take<ab_pair<double>>(nnz);
  ctx->diagA = cv.take<double>(n);
  ctx->diagB = cv.take<double>(n);
  ctx->diagpos = cv.take<int>(n);
  ctx->timer.d_counts = cv.take<int>(kTimerSlots);
  int* sched_dev = cv.take<int>(n);
  ctx->ab32 = cv.take<ab_pair<float>>(nnz);
  ctx->diagA32 = cv.take<float>(n);
  ctx->diagB32 = cv.take<float>(n);
  ctx->static_bytes = cv.off;
  std::vector<float> ab32(2 * (size_t)nnz), dA32(n), dB32(n);
  for (size_t k = 0; k < 2 * (size_t)nnz; ++k) ab32[k] = (float)ab[k];
  for (int64_t i = 0; i < n; ++i) {
    dA32[i] = (float)dA[i];
    dB32[i] = (float)dB[i];
  }
  std::vector<int32_t> order;
  if (band_schedule(n, rp, cl, order)) ctx->sched = sched_dev;
  if (ctx->opt.profile) {
    ctx->events.assign(2 * kTimerSlots, nullptr);
    for (auto& e : ctx->events)
      if (hipEventCreate(&e) != hipSuccess) return bail(SLRF_E_DEVICE, "hipEventCreate failed");
    ctx->timer.events = ctx->events.data();
    ctx->timer.capacity = kTimerSlots;
    launch_fill_zero(ctx->stream, ctx->timer.d_counts, 4 * kTimerSlots);
  }
  hipStream_t s = ctx->stream;
  auto cp = [&](void* dst, const void* src, size_t b) { return hipMemcpyAsync(dst, src, b, hipMemcpyHostToDevice, s); };
  if (cp(ctx->rowptr, rp.data(), 4 * (n + 1)) != hipSuccess || cp(ctx->col, cl.data(), 4 * nnz) != hipSuccess ||
      cp(ctx->ab64, ab.data(), 16 * nnz) != hipSuccess || cp(ctx->diagA, dA.data(), 8 * n) != hipSuccess ||
      cp(ctx->diagB, dB.data(), 8 * n) != hipSuccess || cp(ctx->diagpos, dpos.data(), 4 * n) != hipSuccess ||
      (ctx->sched && cp(ctx->sched, order.data(), 4 * n) != hipSuccess) ||
      cp(ctx->ab32, ab32.data(), 8 * nnz) != hipSuccess || cp(ctx->diagA32, dA32.data(), 4 * n) != hipSuccess ||
      cp(ctx->diagB32, dB32.data(), 4 * n) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
    return bail(SLRF_E_DEVICE, "upload of the merged CSR failed");
  if (ctx->use_ilu) {
    ctx->h_rp = std::move(rp);
    ctx->h_cl = std::move(cl);
    ctx->h_ab = std::move(ab);
    ctx->h_dpos = std::move(dpos);
  }
  *out = ctx;
  return SLRF_OK;
}

void slrf_destroy(slrf_ctx ctx) { delete ctx; }

slrf_status slrf_filter_apply(slrf_ctx ctx, const slrf_poles* poles, int64_t L, const double* d_X, double* d_U,
                              slrf_filter_stats* stats) {
  if (!ctx || !ctx->ws) return SLRF_E_INVALID_ARG;
  if (L < 1 || L > ctx->max_L || !d_X || !d_U || d_X == d_U)
    return fail(ctx, SLRF_E_INVALID_ARG, "bad L or block pointers");
  slrf_status st = check_poles(ctx, poles);
  if (st != SLRF_OK) return st;
  Carver cv{ctx->ws, ctx->static_bytes, ctx->ws_bytes};
  if (ctx->opt.precision == SLRF_MIXED) return filter_mixed(ctx, cv, poles, (int)L, d_X, d_U, stats, ctx->opt.inner_tol);
  return filter_fp64(ctx, cv, poles, (int)L, d_X, d_U, stats);
}

slrf_status slrf_solve_interval(slrf_ctx ctx, double gamma, int64_t L64, const slrf_poles* poles_in,
                                const double* d_V0, int64_t* n_found, double* h_evals, double* d_evecs,
                                double* h_resid, slrf_solve_stats* stats) {
  const double t0 = now_s();
  if (!ctx || !ctx->ws) return SLRF_E_INVALID_ARG;
  if (!(gamma > 0) || L64 < 2 || L64 > ctx->max_L || !n_found || !h_evals || !d_evecs || !h_resid)
    return fail(ctx, SLRF_E_INVALID_ARG, "bad gamma, L or output pointer");
  const int L = (int)L64, n = (int)ctx->n;
  if (L > n) return fail(ctx, SLRF_E_INVALID_ARG, "L exceeds n");
  std::vector<double> psig, pw;
  slrf_poles designed{};
  const slrf_poles* poles = poles_in;
  if (!poles) {
    psig.resize(8);
    pw.resize(8);
    if (slrf_design_poles(4, 1.0, 0.01, gamma, psig.data(), pw.data(), nullptr) != SLRF_OK)
      return fail(ctx, SLRF_E_INVALID_ARG, "pole design failed");
    designed = {4, psig.data(), pw.data()};
    poles = &designed;
  }
  slrf_status st = check_poles(ctx, poles);
  if (st != SLRF_OK) return st;
  hipStream_t s = ctx->stream;
  // outer buffers sit after the Krylov region sized for max_L, max_N
  Carver co{ctx->ws, ctx->static_bytes + krylov_bytes(n, ctx->nnz, ctx->max_L, ctx->max_N, ctx->opt.precision),
            ctx->ws_bytes};
  const int nch = gram_chunks(n, L);
  const int nrr = (n + 255) / 256;
  double* V = co.take<double>((size_t)n * L);
  double* U = co.take<double>((size_t)n * L);
  double* WA = co.take<double>((size_t)n * L);
  double* WB = co.take<double>((size_t)n * L);
  double* X = co.take<double>((size_t)n * L);
  double* part = co.take<double>((size_t)nch * 2 * L * L);
  double* GA = co.take<double>((size_t)L * L);
  double* GB = co.take<double>((size_t)L * L);
  double* Zd = co.take<double>((size_t)L * L);
  double* th_d = co.take<double>(L);
  double* rpart = co.take<double>((size_t)nrr * 2 * L + 2 * L);
  if (co.off > co.cap) return fail(ctx, SLRF_E_WORKSPACE, "workspace too small for the outer iteration");
  if (d_V0)
    HIPCHK(ctx, hipMemcpyAsync(V, d_V0, 8 * (size_t)n * L, hipMemcpyDeviceToDevice, s));
  else
    launch_gaussian(s, (int64_t)n * L, ctx->opt.seed, V);

  slrf_solve_stats ss{};
  std::vector<double> theta, theta2, rho(L, 0.0);
  int prev_count = -1, count = 0;
  double iter_sum = 0, prev_maxr = INFINITY, prev_prev_maxr = INFINITY, mix_c = 1e-3;
  bool converged = false, too_small = false;
  int k = 0;
  for (k = 1; k <= std::max(1, ctx->opt.outer_maxit); ++k) {
    Carver cv{ctx->ws, ctx->static_bytes, ctx->ws_bytes};
    slrf_filter_stats fs{};
    if (ctx->opt.precision == SLRF_MIXED) {
      // Inner accuracy follows the outer residual: target = c * (largest residual
      // of the previous outer iteration), within [1e-13, 1e-4].  The residual of a
      // Ritz pair amplifies the inner error by up to ~lambda_max / theta, so when
      // an outer iteration fails to cut the residual 3x, c shrinks 100x.
      if (prev_prev_maxr < INFINITY && prev_maxr > 0.3 * prev_prev_maxr) mix_c = std::max(1e-9, mix_c * 1e-2);
      const double target = std::max(1e-13, std::min(1e-4, mix_c * prev_maxr));
      st = filter_mixed(ctx, cv, poles, L, V, U, &fs, target);
    } else {
      st = filter_fp64(ctx, cv, poles, L, V, U, &fs);
    }
    if (st != SLRF_OK) return st;
    ss.filter_seconds += fs.seconds;
    ss.spmv_total += fs.spmv;
    iter_sum += fs.mean_iterations;
    ss.kernels.spmm_seconds += fs.spmm_seconds;
    ss.kernels.spmm_launches += fs.spmm_launches;
    ss.kernels.spmm_bytes += fs.spmm_bytes;
    ss.kernels.update_seconds += fs.update_seconds;
    ss.kernels.update_launches += fs.update_launches;
    ss.kernels.update_bytes += fs.update_bytes;
    st = rr_pass(ctx, L, U, X, WA, WB, part, nch, GA, GB, Zd, theta);
    if (st != SLRF_OK) return st;
    st = rr_pass(ctx, L, X, V, WA, WB, part, nch, GA, GB, Zd, theta2);
    if (st != SLRF_OK) return st;
    // residuals of the Ritz pairs (theta2, V)
    launch_spmm_real<double>(s, n, L, ctx->rowptr, ctx->col, ctx->ab64, V, WA, WB);
    HIPCHK(ctx, hipMemcpyAsync(th_d, theta2.data(), 8 * (size_t)L, hipMemcpyHostToDevice, s));
    launch_resid(s, n, L, WA, WB, th_d, rpart, nrr);
    HIPCHK(ctx, hipGetLastError());
    std::vector<double> sums(2 * L);
    HIPCHK(ctx, hipMemcpyAsync(sums.data(), rpart + (size_t)nrr * 2 * L, 16 * (size_t)L, hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    count = 0;
    bool all_ok = true;
    double maxr = 0;
    for (int c = 0; c < L; ++c) {
      rho[c] = std::sqrt(sums[c]) / (std::fabs(theta2[c]) * std::sqrt(sums[L + c]));
      if (theta2[c] > 0 && theta2[c] <= gamma) {
        ++count;
        maxr = std::max(maxr, rho[c]);
        if (!(rho[c] <= ctx->opt.outer_tol)) all_ok = false;
      }
    }
    ss.max_resid = maxr;
    prev_prev_maxr = prev_maxr;
    prev_maxr = count ? maxr : INFINITY;
    if (ctx->verbose)
      fprintf(stderr, "[slrf] outer %d: inner its mean %.1f max %d (rounds %d, maxit %d, breakdown %d, max relres "
                      "%.2e) theta [%.6g, %.6g] count %d max rho %.3e\n",
              k, fs.mean_iterations, fs.max_iterations, fs.refinements, fs.n_maxit, fs.n_breakdown, fs.max_relres,
              theta2[0], theta2[L - 1], count, maxr);
    if (count == L) {
      too_small = true;
      break;
    }
    if (count == prev_count && all_ok) {
      converged = true;
      break;
    }
    prev_count = count;
  }
  ss.outer_iterations = std::min(k, std::max(1, ctx->opt.outer_maxit));
  ss.inner_iterations = iter_sum / std::max(1, ss.outer_iterations);
  HIPCHK(ctx, hipMemcpyAsync(d_evecs, V, 8 * (size_t)n * L, hipMemcpyDeviceToDevice, s));
  HIPCHK(ctx, hipStreamSynchronize(s));
  int found = 0;
  for (int c = 0; c < L; ++c) {
    h_evals[c] = theta2[c];
    h_resid[c] = rho[c];
    if (theta2[c] > 0 && theta2[c] <= gamma && rho[c] <= ctx->opt.outer_tol) ++found;
  }
  *n_found = found;
  ss.n_found = found;
  ss.seconds = now_s() - t0;
  if (stats) *stats = ss;
  if (too_small) return fail(ctx, SLRF_E_SUBSPACE_TOO_SMALL, "all L Ritz values lie in (0, gamma]: increase L");
  if (!converged) return fail(ctx, SLRF_E_NOT_CONVERGED, "outer iteration limit reached");
  return SLRF_OK;
}

}  // extern "C"

extern "C" {

size_t slrf_test_gram_scratch(int64_t n, int64_t L) {
  return (size_t)gram_chunks((int)n, (int)L) * 2 * L * L * sizeof(double);
}

int slrf_test_gram(int64_t n, int64_t L, const double* U, const double* WA, const double* WB, double* GA,
                   double* GB, void* scratch, size_t scratch_bytes, void* hip_stream) {
  if (n < 1 || L < 1 || !U || !WA || !WB || !GA || !GB || scratch_bytes < slrf_test_gram_scratch(n, L))
    return SLRF_E_INVALID_ARG;
  hipStream_t s = (hipStream_t)hip_stream;
  launch_gram(s, (int)n, (int)L, U, WA, WB, (double*)scratch, gram_chunks((int)n, (int)L), GA, GB);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) return SLRF_E_DEVICE;
  return SLRF_OK;
}

int slrf_test_gemm(int64_t n, int64_t L, int64_t r, const double* X, const double* Z, double* Y,
                   void* hip_stream) {
  if (n < 1 || L < 1 || r < 1 || !X || !Z || !Y) return SLRF_E_INVALID_ARG;
  hipStream_t s = (hipStream_t)hip_stream;
  const double* xs[1] = {X};
  double* ys[1] = {Y};
  launch_gemm_nz(s, (int)n, (int)L, (int)r, 1, xs, Z, ys);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) return SLRF_E_DEVICE;
  return SLRF_OK;
}

}  // extern "C"

// Per-pencil kernels of the SLRF eigensolver (gfx950): shifted-operator
// diagonals, filter sum, real products with the merged pencil, FP64 MFMA Gram
// and Ritz-update products, residual norms, start block.  Every dense block is
// row-major (n, L) float64; the batched Krylov kernels are in krylov.hip.
#include "device_util.h"

#include <algorithm>

namespace slrf {


// v = diag(A) - sigma_j diag(B); d = cd v, dinv = ci / v (cd = ci = 1: the
// Jacobi diagonal and its inverse)
template <typename R>
__global__ void k_jacobi(int n, int N, const R* dA, const R* dB, const cx<R>* sigma, cx<R>* d,
                         cx<R>* dinv, R cd, R ci) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * N) return;
  const int i = (int)(e / N), j = (int)(e % N);
  const cx<R> s = sigma[j];
  const cx<R> v = {dA[i] - s.re * dB[i], -s.im * dB[i]};
  d[e] = {cd * v.re, cd * v.im};
  dinv[e] = cdiv(cx<R>{ci, 0}, v);
}
template <typename R>
void launch_jacobi_diag(hipStream_t s, int n, int N, const R* diagA, const R* diagB,
                        const cx<R>* sigma, cx<R>* d, cx<R>* dinv, double cd, double ci) {
  const int64_t tot = (int64_t)n * N;
  k_jacobi<R><<<dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s>>>(n, N, diagA, diagB, sigma, d, dinv,
                                                                        (R)cd, (R)ci);
}

// U[i, l] (+)= sum_j 2 Re(w_j x[i, col_of(j, l)])
template <typename R>
__global__ void k_filter_sum(int n, int L, int N, int W, int rmaj, const cx<R>* __restrict__ x,
                             const double* __restrict__ w, double* __restrict__ U, int accumulate) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * L) return;
  const int64_t i = e / L;
  const int l = (int)(e % L);
  double s = accumulate ? U[e] : 0.0;
  for (int j = 0; j < N; ++j) {
    const int c = col_of(j, l, L, N, rmaj);  // tile c / W is an n x W panel
    const cx<R> y = x[(int64_t)(c / W) * n * W + i * W + c % W];
    s += 2.0 * (w[2 * j] * (double)y.re - w[2 * j + 1] * (double)y.im);
  }
  U[e] = s;
}
template <typename R>
void launch_filter_sum(hipStream_t s, int n, int L, int N, int W, int rmaj, const cx<R>* x, const double* w,
                       double* U, bool accumulate) {
  const int64_t tot = (int64_t)n * L;
  k_filter_sum<R><<<dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s>>>(n, L, N, W, rmaj, x, w, U,
                                                                             accumulate ? 1 : 0);
}

// Real products of the merged pencil with a real block: one wavefront per row.
template <typename R>
__global__ __launch_bounds__(WG) void k_spmm_real(int n, int L, const int* __restrict__ rowptr,
                                                 const int* __restrict__ col,
                                                 const ab_pair<R>* __restrict__ ab,
                                                 const double* __restrict__ X, double* __restrict__ AX,
                                                 double* __restrict__ BX) {
  const int row = blockIdx.x * 4 + wave_id();
  if (row >= n) return;
  const int lane = lane_id();
  const int k0 = rowptr[row], k1 = rowptr[row + 1];
  for (int c = lane; c < L; c += WAVE) {
    double sa = 0, sb = 0;
    for (int k = k0; k < k1; ++k) {
      const int j = col[k];
      const ab_pair<R> m = ab[k];
      const double x = X[(size_t)j * L + c];
      sa += (double)m.a * x;
      sb += (double)m.b * x;
    }
    if (AX) AX[(size_t)row * L + c] = sa;
    if (BX) BX[(size_t)row * L + c] = sb;
  }
}
template <typename R>
void launch_spmm_real(hipStream_t s, int n, int L, const int* rowptr, const int* col, const ab_pair<R>* ab,
                      const double* X, double* AX, double* BX) {
  k_spmm_real<R><<<dim3((n + 3) / 4), dim3(WG), 0, s>>>(n, L, rowptr, col, ab, X, AX, BX);
}

// ---------------------------------------------------------------------------
// FP64 MFMA (v_mfma_f64_16x16x4_f64).  Operand layout for D(16x16) += A(16x4) B(4x16):
// lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]; it receives
// D[l / 16 + 4 q][l % 16] in accumulator element q (checked on gfx950 with
// indicator inputs).
typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// FP32 variant: v_mfma_f32_16x16x4f32 (FP32 inputs, FP32 accumulation), used
// for the Gram products of the first of the two projections while the Ritz
// pairs are still far from converged.  Its 16 x 16 accumulator puts row 4 (l / 16) + q, column l % 16 in
// lane l's element q (the FP64 instruction: row l / 16 + 4 q).
typedef float f4 __attribute__((ext_vector_type(4)));

template <bool F32>
struct Mfma;
template <>
struct Mfma<false> {
  using acc_t = d4;
  using in_t = double;
  static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) { return mfma64(a, b, c); }
  static __device__ __forceinline__ int row(int li, int q) { return li + 4 * q; }
};
template <>
struct Mfma<true> {
  using acc_t = f4;
  using in_t = float;
  static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int li, int q) { return 4 * li + q; }
};

// Partial Gram matrices over a chunk of rows: GA = U^T WA, GB = U^T WB.
// A workgroup covers a 128 (rows of G) x 64 (columns of G) region; wavefront w
// covers 64 x 32 of it as 4 x 2 tiles of 16 x 16, for both products.  F32: the
// FP64 inputs are rounded to FP32 as they are loaded.
template <bool F32>
__global__ __launch_bounds__(WG) void k_gram(int n, int L, const double* __restrict__ U,
                                            const double* __restrict__ WA, const double* __restrict__ WB,
                                            int rows_per_chunk, double* __restrict__ part) {
  using M = Mfma<F32>;
  using T = typename M::in_t;
  const int chunk = blockIdx.x;
  const int nbb = (L + 63) / 64;
  const int ba = blockIdx.y / nbb, bb = blockIdx.y % nbb;
  const int w = wave_id(), lane = lane_id();
  const int a0 = ba * 128 + (w >> 1) * 64;
  const int b0 = bb * 64 + (w & 1) * 32;
  const int li = lane >> 4, lj = lane & 15;
  typename M::acc_t accA[4][2], accB[4][2];
#pragma unroll
  for (int ta = 0; ta < 4; ++ta)
#pragma unroll
    for (int tb = 0; tb < 2; ++tb) {
      accA[ta][tb] = typename M::acc_t{0, 0, 0, 0};
      accB[ta][tb] = typename M::acc_t{0, 0, 0, 0};
    }
  const int i0 = chunk * rows_per_chunk;
  const int i1 = min(n, i0 + rows_per_chunk);
  for (int i = i0; i < i1; i += 4) {
    const int row = i + li;
    const bool rv = row < i1;
    T a[4], xa[2], xb[2];
#pragma unroll
    for (int ta = 0; ta < 4; ++ta) {
      const int cidx = a0 + 16 * ta + lj;
      a[ta] = (T)((rv && cidx < L) ? U[(size_t)row * L + cidx] : 0.0);
    }
#pragma unroll
    for (int tb = 0; tb < 2; ++tb) {
      const int cidx = b0 + 16 * tb + lj;
      const bool ok = rv && cidx < L;
      xa[tb] = (T)(ok ? WA[(size_t)row * L + cidx] : 0.0);
      xb[tb] = (T)(ok ? WB[(size_t)row * L + cidx] : 0.0);
    }
#pragma unroll
    for (int ta = 0; ta < 4; ++ta)
#pragma unroll
      for (int tb = 0; tb < 2; ++tb) {
        accA[ta][tb] = M::op(a[ta], xa[tb], accA[ta][tb]);
        accB[ta][tb] = M::op(a[ta], xb[tb], accB[ta][tb]);
      }
  }
  const size_t LL = (size_t)L * L;
  double* pA = part + (size_t)chunk * 2 * LL;
  double* pB = pA + LL;
#pragma unroll
  for (int ta = 0; ta < 4; ++ta)
#pragma unroll
    for (int tb = 0; tb < 2; ++tb)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int ga = a0 + 16 * ta + M::row(li, q);
        const int gb = b0 + 16 * tb + lj;
        if (ga < L && gb < L) {
          pA[(size_t)ga * L + gb] = (double)accA[ta][tb][q];
          pB[(size_t)ga * L + gb] = (double)accB[ta][tb][q];
        }
      }
}

__global__ void k_gram_reduce(int L, int nchunks, const double* __restrict__ part, double* __restrict__ GA,
                              double* __restrict__ GB) {
  const size_t LL = (size_t)L * L;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 2 * LL) return;
  const int which = (int)(e / LL);
  const size_t o = e % LL;
  double s = 0;
  for (int c = 0; c < nchunks; ++c) s += part[(size_t)c * 2 * LL + which * LL + o];
  (which ? GB : GA)[o] = s;
}

// Row chunks of the split-K Gram product: independent of L so that the partial
// buffer sized for the largest L also fits every smaller L.
int gram_chunks(int n, int /*L*/) {
  int rows = (n + 255) / 256;
  rows = std::max(64, (rows + 3) / 4 * 4);
  return (n + rows - 1) / rows;
}

void launch_gram(hipStream_t s, int n, int L, const double* U, const double* WA, const double* WB,
                 double* part, int nchunks, double* GA, double* GB, bool f32) {
  int rows = (n + nchunks - 1) / nchunks;
  rows = (rows + 3) / 4 * 4;
  const int tiles = ((L + 127) / 128) * ((L + 63) / 64);
  if (f32)
    k_gram<true><<<dim3(nchunks, tiles), dim3(WG), 0, s>>>(n, L, U, WA, WB, rows, part);
  else
    k_gram<false><<<dim3(nchunks, tiles), dim3(WG), 0, s>>>(n, L, U, WA, WB, rows, part);
  const size_t tot = 2 * (size_t)L * L;
  k_gram_reduce<<<dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s>>>(L, nchunks, part, GA, GB);
}

// Y_b = X_b Z : (n x L)(L x r).  Wavefront w of workgroup bx owns rows
// [64 bx + 16 w, +16) and sweeps the output columns in groups of 8 tiles.
struct GemmBlocks {
  const double* X[3];
  double* Y[3];
};

__global__ __launch_bounds__(WG) void k_gemm_nz(int n, int L, int r, GemmBlocks gb,
                                               const double* __restrict__ Z) {
  using M = Mfma<false>;
  using T = typename M::in_t;
  const double* __restrict__ X = gb.X[blockIdx.y];
  double* __restrict__ Y = gb.Y[blockIdx.y];
  const int w = wave_id(), lane = lane_id();
  const int li = lane >> 4, lj = lane & 15;
  const int row0 = blockIdx.x * 64 + w * 16;
  if (row0 >= n) return;
  for (int c0 = 0; c0 < r; c0 += 128) {
    typename M::acc_t acc[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) acc[t] = typename M::acc_t{0, 0, 0, 0};
    for (int k0 = 0; k0 < L; k0 += 4) {
      const int row = row0 + lj;
      const int k = k0 + li;
      const T a = (T)((row < n && k < L) ? X[(size_t)row * L + k] : 0.0);
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int cc = c0 + 16 * t + lj;
        const T b = (T)((k < L && cc < r) ? Z[(size_t)k * r + cc] : 0.0);
        acc[t] = M::op(a, b, acc[t]);
      }
    }
#pragma unroll
    for (int t = 0; t < 8; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = row0 + M::row(li, q);
        const int cc = c0 + 16 * t + lj;
        if (row < n && cc < r) Y[(size_t)row * r + cc] = (double)acc[t][q];
      }
  }
}

void launch_gemm_nz(hipStream_t s, int n, int L, int r, int nb, const double* const* X, const double* Z,
                    double* const* Y) {
  GemmBlocks gbk{};
  for (int b = 0; b < nb; ++b) {
    gbk.X[b] = X[b];
    gbk.Y[b] = Y[b];
  }
  k_gemm_nz<<<dim3((n + 63) / 64, nb), dim3(WG), 0, s>>>(n, L, r, gbk, Z);
}

// Warm start of the shifted solves: Y0 = Y_prev C per pole, with the real L x L
// C = X_prev^T B X_new (row-major, C[l * L + l']).  Y_prev, Y0: tile-major
// complex FP64 blocks (tiles of W columns) in column order rmaj, K = N L
// columns padded to Kp; the padding columns of Y0 are zero.  On FP64 MFMA: for
// pole j the rows (i, re) and (i, im) of Y_prev's columns of that pole form a
// 2n x L real matrix A_j, and Y0's columns of pole j are A_j C.  A wavefront
// owns 16 rows of A_j (8 grid rows, both parts) and sweeps the output columns
// 128 at a time; the pole-0 wavefronts also zero their rows' padding columns.
__global__ __launch_bounds__(WG) void k_recycle(int n, int L, int N, int W, int Kp, int rmaj,
                                               const double* __restrict__ Yp, const double* __restrict__ C,
                                               double* __restrict__ Y0) {
  using M = Mfma<false>;
  const int j = blockIdx.y;
  const int w = wave_id(), lane = lane_id();
  const int li = lane >> 4, lj = lane & 15;
  const int64_t rows = 2 * (int64_t)n;
  const int64_t row0 = (int64_t)blockIdx.x * 64 + w * 16;
  if (row0 >= rows) return;
  // index (in doubles) of A_j[r][l]: grid row r / 2, part r % 2, column l of pole j
  auto elem = [&](int64_t r, int l) -> int64_t {
    const int c = col_of(j, l, L, N, rmaj);
    return (((int64_t)(c / W) * n + (r >> 1)) * W + c % W) * 2 + (r & 1);
  };
  const int64_t ra = row0 + lj;
  const bool rok = ra < rows;
  for (int c0 = 0; c0 < L; c0 += 128) {
    M::acc_t acc[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) acc[t] = M::acc_t{0, 0, 0, 0};
    for (int k0 = 0; k0 < L; k0 += 4) {
      const int k = k0 + li;
      const double a = (rok && k < L) ? Yp[elem(ra, k)] : 0.0;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int cc = c0 + 16 * t + lj;
        const double bv = (k < L && cc < L) ? C[(int64_t)k * L + cc] : 0.0;
        acc[t] = M::op(a, bv, acc[t]);
      }
    }
#pragma unroll
    for (int t = 0; t < 8; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t r = row0 + M::row(li, q);
        const int cc = c0 + 16 * t + lj;
        if (r < rows && cc < L) Y0[elem(r, cc)] = acc[t][q];
      }
  }
  const int pad = Kp - N * L;
  if (j == 0 && pad > 0) {
    const int64_t i0 = row0 >> 1;
    for (int e = lane; e < 8 * pad; e += WAVE) {
      const int64_t i = i0 + e / pad;
      const int c = N * L + e % pad;
      if (i < n) {
        const int64_t o = (((int64_t)(c / W) * n + i) * W + c % W) * 2;
        Y0[o] = 0.0;
        Y0[o + 1] = 0.0;
      }
    }
  }
}

void launch_recycle(hipStream_t s, int n, int L, int N, int W, int Kp, int rmaj, const cx<double>* Yp,
                    const double* C, cx<double>* Y0) {
  const unsigned blocks = (unsigned)((2 * (int64_t)n + 63) / 64);
  k_recycle<<<dim3(blocks, (unsigned)N), dim3(WG), 0, s>>>(n, L, N, W, Kp, rmaj, (const double*)Yp, C,
                                                            (double*)Y0);
}

// Residual column sums over row blocks of 256 rows.
__global__ __launch_bounds__(WG) void k_resid(int n, int L, const double* __restrict__ AX,
                                             const double* __restrict__ BX, const double* __restrict__ theta,
                                             double* __restrict__ part) {
  const int w = wave_id(), lane = lane_id();
  const int r0 = blockIdx.x * 256, r1 = min(n, r0 + 256);
  __shared__ double red[2][4][WAVE];
  for (int c0 = 0; c0 < L; c0 += WAVE) {
    const int c = c0 + lane;
    double rr = 0, bb = 0;
    if (c < L) {
      const double th = theta[c];
      for (int i = r0 + w; i < r1; i += 4) {
        const double b = BX[(size_t)i * L + c];
        const double d = AX[(size_t)i * L + c] - th * b;
        rr += d * d;
        bb += b * b;
      }
    }
    red[0][w][lane] = rr;
    red[1][w][lane] = bb;
    __syncthreads();
    if (w == 0 && c < L) {
      part[((size_t)blockIdx.x * 2 + 0) * L + c] = red[0][0][lane] + red[0][1][lane] + red[0][2][lane] + red[0][3][lane];
      part[((size_t)blockIdx.x * 2 + 1) * L + c] = red[1][0][lane] + red[1][1][lane] + red[1][2][lane] + red[1][3][lane];
    }
    __syncthreads();
  }
}

__global__ void k_resid_reduce(int L, int nrb, double* part) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 2 * L) return;
  const int which = e / L, c = e % L;
  double s = 0;
  for (int b = 0; b < nrb; ++b) s += part[((size_t)b * 2 + which) * L + c];
  // the reduced sums go after the per-block partials
  part[(size_t)nrb * 2 * L + e] = s;
}

void launch_resid(hipStream_t s, int n, int L, const double* AX, const double* BX, const double* theta,
                  double* part, int nrb) {
  k_resid<<<dim3(nrb), dim3(WG), 0, s>>>(n, L, AX, BX, theta, part);
  k_resid_reduce<<<dim3((2 * L + 255) / 256), dim3(256), 0, s>>>(L, nrb, part);
}

// SplitMix64 + Box-Muller, element e of the stream for `seed`
__device__ __forceinline__ uint64_t splitmix(uint64_t seed, uint64_t idx) {
  uint64_t z = seed + (idx + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__global__ void k_gaussian(int64_t count, uint64_t seed, double* out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  const int64_t pair = e >> 1;
  const double u1 = ((double)(splitmix(seed, 2 * pair) >> 11) + 1.0) * 0x1.0p-53;
  const double u2 = ((double)(splitmix(seed, 2 * pair + 1) >> 11) + 1.0) * 0x1.0p-53;
  const double r = sqrt(-2.0 * log(u1));
  const double t = 6.283185307179586476925 * u2;
  out[e] = (e & 1) ? r * sin(t) : r * cos(t);
}
void launch_gaussian(hipStream_t s, int64_t count, uint64_t seed, double* out) {
  k_gaussian<<<dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s>>>(count, seed, out);
}

__global__ void k_fill_zero(uint32_t* p, size_t words) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < words) p[e] = 0;
}
void launch_fill_zero(hipStream_t s, void* p, size_t bytes) {
  const size_t words = bytes / 4;
  if (words) k_fill_zero<<<dim3((unsigned)((words + 255) / 256)), dim3(256), 0, s>>>((uint32_t*)p, words);
}

// explicit instantiations
#define SLRF_INST(R)                                                                                          \
  template void launch_jacobi_diag<R>(hipStream_t, int, int, const R*, const R*, const cx<R>*, cx<R>*,     \
                                      cx<R>*, double, double);                                              \
  template void launch_filter_sum<R>(hipStream_t, int, int, int, int, int, const cx<R>*, const double*,   \
                                     double*, bool);                                                        \
  template void launch_spmm_real<R>(hipStream_t, int, int, const int*, const int*, const ab_pair<R>*,      \
                                    const double*, double*, double*);
SLRF_INST(double)
SLRF_INST(float)

}  // namespace slrf

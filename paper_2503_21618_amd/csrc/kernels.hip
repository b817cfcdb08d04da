// gfx950 kernels of the SLRF eigensolver.
//
// Layout in HBM: every dense block is row-major.  The Krylov state of all
// N poles x L columns is one (n, K) complex block, K = N * L, column
// c = j * L + l belongs to pole j and right-hand side l; complex numbers are
// (re, im) interleaved, so one row of a 64-column tile is a contiguous
// 64 * sizeof(cx<R>) byte segment (1 KiB in FP64).
//
// Work decomposition shared by all Krylov kernels: a grid of G workgroups of
// 256 threads (4 wavefronts of 64) sweeps the 64-column tiles one after the
// other; within a tile each lane owns one column and each wavefront walks every
// 4th row of its row blocks (see WgPos for how rows are assigned per XCD).
// Per-column dot products therefore accumulate in registers with no cross-lane
// traffic; the 4 wavefronts are combined through LDS and the G workgroups by a
// per-column kernel that sums [G][K] partials in a fixed order (bitwise
// reproducible).
#include "kernels.h"

#include <algorithm>

namespace slrf {

constexpr int WAVE = 64;
constexpr int WG = 256;
constexpr int kWgPerXcd = 128;  // workgroups per XCD in the Krylov kernels

__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }
__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t padded) {
  const int64_t per = padded >> 3;
  return (bid & 7) * per + (bid >> 3);
}

template <typename R>
__device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__device__ __forceinline__ cx<R> cadd(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__device__ __forceinline__ cx<R> csub(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__device__ __forceinline__ cx<R> cdiv(cx<R> a, cx<R> b) {
  // Smith's algorithm
  if (fabs(b.re) >= fabs(b.im)) {
    R q = b.im / b.re, den = b.re + b.im * q;
    return {(a.re + a.im * q) / den, (a.im - a.re * q) / den};
  }
  R q = b.re / b.im, den = b.re * q + b.im;
  return {(a.re * q + a.im) / den, (a.im * q - a.re) / den};
}

KGeom make_geom(int n, int N, int L, int rows_per_block) {
  KGeom g;
  g.n = n;
  g.N = N;
  g.L = L;
  g.K = N * L;
  g.rows_per_block = rows_per_block;
  g.nrb = (n + rows_per_block - 1) / rows_per_block;
  g.nct = (g.K + WAVE - 1) / WAVE;
  g.slab = (g.nrb + 7) / 8;
  const int per_xcd = std::max(1, std::min(kWgPerXcd, g.slab));
  g.G = 8 * per_xcd;
  g.steps = (g.slab + per_xcd - 1) / per_xcd;
  g.sched = nullptr;
  return g;
}

// Workgroup b runs on XCD b % 8 (round-robin dispatch).  XCD x owns the
// contiguous slab of row blocks [x * slab, (x + 1) * slab); its per_xcd
// workgroups advance through the slab together, step t covering row blocks
// x * slab + t * per_xcd + [0, per_xcd), so the rows in flight on one XCD stay
// within about one grid plane and the neighbours gathered by the sparse product
// are re-read from that XCD's L2 instead of HBM.
struct WgPos {
  int x, q, per, lane, w;
};

__device__ __forceinline__ WgPos wg_pos(const KGeom& g) {
  WgPos p;
  p.x = blockIdx.x & 7;
  p.q = blockIdx.x >> 3;
  p.per = g.G >> 3;
  p.lane = lane_id();
  p.w = wave_id();
  return p;
}

// row block of step t for this workgroup, or -1 once past the slab
__device__ __forceinline__ int step_block(const KGeom& g, const WgPos& p, int t) {
  const int j = t * p.per + p.q;
  if (j >= g.slab) return -1;
  const int rb = p.x * g.slab + j;
  return rb < g.nrb ? rb : -1;
}

// true if any column of the 64-column tile is in one of the given states
__device__ __forceinline__ bool tile_has(const int* flags, int c, bool valid, int s0, int s1) {
  const int f = valid ? flags[c] : -1;
  return __any(f == s0 || f == s1);
}

// one vector atomic per processed (workgroup, tile) when instrumented
__device__ __forceinline__ void count_tile(int* counter) {
  if (counter && threadIdx.x == 0) atomicAdd(counter, 1);
}

// Sum of the 4 wavefronts' per-lane values in a fixed order; lane c of wave 0
// stores it at out[c] (out points at this workgroup's slice of the tile).
template <typename T>
__device__ __forceinline__ void wg_store_partial(T v, int w, int lane, bool valid, T* out) {
  __shared__ T red[4][WAVE];
  red[w][lane] = v;
  __syncthreads();
  if (w == 0 && valid) out[lane] = red[0][lane] + red[1][lane] + red[2][lane] + red[3][lane];
  __syncthreads();
}

template <typename R>
__device__ __forceinline__ void wg_store_partial_cx(cx<R> v, int w, int lane, bool valid, cx<R>* out) {
  __shared__ R rr[4][WAVE], ri[4][WAVE];
  rr[w][lane] = v.re;
  ri[w][lane] = v.im;
  __syncthreads();
  if (w == 0 && valid)
    out[lane] = {rr[0][lane] + rr[1][lane] + rr[2][lane] + rr[3][lane],
                 ri[0][lane] + ri[1][lane] + ri[2][lane] + ri[3][lane]};
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Complex-shifted sparse product over the merged CSR:
//   Q[i, c] = sum_j (a_ij - sigma_c b_ij) P[j, c]
// (A - sigma B is never formed: each (a, b) pair is read once per tile and the
// pole of the column is applied when the row is finished.)
// The row's entries are taken in chunks of CH: CH (col, a, b) entries are read
// (wave-uniform, scalar loads), then CH gathers are issued back to back with no
// branches, then the FMAs.  Entries past the row end repeat the last valid
// column with zero coefficients, and lanes past K read column K-1 (both stay in
// bounds; their contributions are discarded).
template <typename R, int CH>
__device__ __forceinline__ cx<R> shifted_row(int i, const int* __restrict__ rowptr,
                                             const int* __restrict__ col,
                                             const ab_pair<R>* __restrict__ ab,
                                             const cx<R>* __restrict__ Pc, int K, cx<R> sig) {
  const int k0 = rowptr[i], k1 = rowptr[i + 1];
  R apr = 0, api = 0, bpr = 0, bpi = 0;
  for (int kb = k0; kb < k1; kb += CH) {
    int jj[CH];
    ab_pair<R> m[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int k = min(kb + u, k1 - 1);
      jj[u] = col[k];
      m[u] = ab[k];
      if (kb + u >= k1) m[u] = ab_pair<R>{0, 0};
    }
    cx<R> x[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u) x[u] = Pc[(size_t)jj[u] * K];
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      apr += m[u].a * x[u].re;
      api += m[u].a * x[u].im;
      bpr += m[u].b * x[u].re;
      bpi += m[u].b * x[u].im;
    }
  }
  return {apr - (sig.re * bpr - sig.im * bpi), api - (sig.re * bpi + sig.im * bpr)};
}

constexpr int kChunk = 16;

// v = S p_hat, partial (rhat, v)
template <typename R>
__global__ __launch_bounds__(WG) void k_spmm_v(KGeom g, KrylovState<R> st, const int* __restrict__ rowptr,
                                              const int* __restrict__ col,
                                              const ab_pair<R>* __restrict__ ab, int* counter) {
  const WgPos p = wg_pos(g);
  for (int ct = 0; ct < g.nct; ++ct) {
    const int c = ct * WAVE + p.lane;
    const bool valid = c < g.K;
    const int cc = min(c, g.K - 1);
    R dr = 0, di = 0;
    if (tile_has(st.flags, c, valid, COL_ACTIVE, COL_ACTIVE)) {
      count_tile(counter);
      const cx<R> sig = st.sigma_col[cc];
      const int l = cc % g.L;
      for (int t = 0; t < g.steps; ++t) {
        const int rb = step_block(g, p, t);
        if (rb < 0) break;
        const int r1 = min((rb + 1) * g.rows_per_block, g.n);
        for (int pos = rb * g.rows_per_block + p.w; pos < r1; pos += 4) {
          const int i = g.sched ? g.sched[pos] : pos;
          const cx<R> q = shifted_row<R, kChunk>(i, rowptr, col, ab, st.ph + cc, g.K, sig);
          if (valid) {
            st.v[(size_t)i * g.K + c] = q;
            if (st.rhat_cx) {  // conj(rhat) * v
              const cx<R> rh = st.rhat_cx[(size_t)i * g.K + c];
              dr += rh.re * q.re + rh.im * q.im;
              di += rh.re * q.im - rh.im * q.re;
            } else {
              const R rh = st.rhat[(size_t)i * g.L + l];
              dr += rh * q.re;
              di += rh * q.im;
            }
          }
        }
      }
    }
    wg_store_partial_cx<R>({dr, di}, p.w, p.lane, valid, st.part_a + (size_t)blockIdx.x * g.K + ct * WAVE);
  }
}

// t = S s_hat, partials (t, s) = t^H s and (t, t)
template <typename R>
__global__ __launch_bounds__(WG) void k_spmm_t(KGeom g, KrylovState<R> st, const int* __restrict__ rowptr,
                                              const int* __restrict__ col,
                                              const ab_pair<R>* __restrict__ ab, int* counter) {
  const WgPos p = wg_pos(g);
  for (int ct = 0; ct < g.nct; ++ct) {
    const int c = ct * WAVE + p.lane;
    const bool valid = c < g.K;
    const int cc = min(c, g.K - 1);
    R tsr = 0, tsi = 0, tt = 0;
    if (tile_has(st.flags, c, valid, COL_ACTIVE, COL_ACTIVE)) {
      count_tile(counter);
      const cx<R> sig = st.sigma_col[cc];
      const int pole = cc / g.L;
      for (int t = 0; t < g.steps; ++t) {
        const int rb = step_block(g, p, t);
        if (rb < 0) break;
        const int r1 = min((rb + 1) * g.rows_per_block, g.n);
        for (int pos = rb * g.rows_per_block + p.w; pos < r1; pos += 4) {
          const int i = g.sched ? g.sched[pos] : pos;
          const cx<R> tv = shifted_row<R, kChunk>(i, rowptr, col, ab, st.sh + cc, g.K, sig);
          if (valid) {
            const size_t e = (size_t)i * g.K + c;
            st.t[e] = tv;
            const cx<R> s = st.s ? st.s[e] : cmul(st.d[(size_t)i * g.N + pole], st.sh[e]);
            tsr += tv.re * s.re + tv.im * s.im;  // conj(t) * s
            tsi += tv.re * s.im - tv.im * s.re;
            tt += tv.re * tv.re + tv.im * tv.im;
          }
        }
      }
    }
    const size_t o = (size_t)blockIdx.x * g.K + ct * WAVE;
    wg_store_partial_cx<R>({tsr, tsi}, p.w, p.lane, valid, st.part_a + o);
    wg_store_partial<R>(tt, p.w, p.lane, valid, st.part_b + o);
  }
}

// p = r + beta (p - omega v)  (first iteration: p = r).
// Jacobi: p itself is not stored; p_hat = p / d with p = d p_hat.
// General preconditioner: p is stored and p_hat is formed by the preconditioner.
template <typename R>
__global__ __launch_bounds__(WG) void k_update_p(KGeom g, KrylovState<R> st, int first, int* counter) {
  const WgPos p = wg_pos(g);
  for (int ct = 0; ct < g.nct; ++ct) {
    const int c = ct * WAVE + p.lane;
    const bool valid = c < g.K;
    if (!tile_has(st.flags, c, valid, COL_ACTIVE, COL_ACTIVE)) continue;
    count_tile(counter);
    if (!valid || st.flags[c] != COL_ACTIVE) continue;
    const int pole = c / g.L;
    const cx<R> beta = st.beta[c], omega = st.omega[c];
    for (int t = 0; t < g.steps; ++t) {
      const int rb = step_block(g, p, t);
      if (rb < 0) break;
      const int r1 = min((rb + 1) * g.rows_per_block, g.n);
      for (int i = rb * g.rows_per_block + p.w; i < r1; i += 4) {
        const size_t e = (size_t)i * g.K + c;
        cx<R> pn = st.r[e];
        if (st.p) {
          if (!first) pn = cadd(pn, cmul(beta, csub(st.p[e], cmul(omega, st.v[e]))));
          st.p[e] = pn;
        } else {
          const cx<R> di = st.dinv[(size_t)i * g.N + pole];
          if (!first) {
            const cx<R> dd = st.d[(size_t)i * g.N + pole];
            pn = cadd(pn, cmul(beta, csub(cmul(dd, st.ph[e]), cmul(omega, st.v[e]))));
          }
          st.ph[e] = cmul(pn, di);
        }
      }
    }
  }
}

// s = r - alpha v (Jacobi: s_hat = s / d is stored instead) ; partial |s|^2
template <typename R>
__global__ __launch_bounds__(WG) void k_update_s(KGeom g, KrylovState<R> st, int* counter) {
  const WgPos p = wg_pos(g);
  for (int ct = 0; ct < g.nct; ++ct) {
    const int c = ct * WAVE + p.lane;
    const bool valid = c < g.K;
    R ss = 0;
    if (tile_has(st.flags, c, valid, COL_ACTIVE, COL_ACTIVE)) {
      count_tile(counter);
      if (valid && st.flags[c] == COL_ACTIVE) {
        const int pole = c / g.L;
        const cx<R> alpha = st.alpha[c];
        for (int t = 0; t < g.steps; ++t) {
          const int rb = step_block(g, p, t);
          if (rb < 0) break;
          const int r1 = min((rb + 1) * g.rows_per_block, g.n);
          for (int i = rb * g.rows_per_block + p.w; i < r1; i += 4) {
            const size_t e = (size_t)i * g.K + c;
            const cx<R> s = csub(st.r[e], cmul(alpha, st.v[e]));
            ss += s.re * s.re + s.im * s.im;
            if (st.s)
              st.s[e] = s;
            else
              st.sh[e] = cmul(s, st.dinv[(size_t)i * g.N + pole]);
          }
        }
      }
    }
    wg_store_partial<R>(ss, p.w, p.lane, valid, st.part_b + (size_t)blockIdx.x * g.K + ct * WAVE);
  }
}

// x += alpha p_hat + omega s_hat ; r = s - omega t ; partials (rhat, r), |r|^2
// Columns that converged at the half step take x += alpha p_hat only.
template <typename R>
__global__ __launch_bounds__(WG) void k_update_x(KGeom g, KrylovState<R> st, int first, int* counter) {
  const WgPos p = wg_pos(g);
  for (int ct = 0; ct < g.nct; ++ct) {
    const int c = ct * WAVE + p.lane;
    const bool valid = c < g.K;
    R rr = 0, ri = 0, nn = 0;
    if (tile_has(st.flags, c, valid, COL_ACTIVE, COL_HALF_PENDING)) {
      count_tile(counter);
      const int f = valid ? st.flags[c] : -1;
      const bool act = f == COL_ACTIVE, half = f == COL_HALF_PENDING;
      if (act || half) {
        const int pole = c / g.L;
        const int l = c % g.L;
        const cx<R> alpha = st.alpha[c];
        const cx<R> omega = act ? st.omega[c] : cx<R>{0, 0};
        for (int t = 0; t < g.steps; ++t) {
          const int rb = step_block(g, p, t);
          if (rb < 0) break;
          const int r1 = min((rb + 1) * g.rows_per_block, g.n);
          for (int i = rb * g.rows_per_block + p.w; i < r1; i += 4) {
            const size_t e = (size_t)i * g.K + c;
            cx<R> x = first ? cx<R>{0, 0} : st.x[e];
            x = cadd(x, cmul(alpha, st.ph[e]));
            if (act) {
              const cx<R> sh = st.sh[e];
              x = cadd(x, cmul(omega, sh));
              const cx<R> sv = st.s ? st.s[e] : cmul(st.d[(size_t)i * g.N + pole], sh);
              const cx<R> r = csub(sv, cmul(omega, st.t[e]));
              st.r[e] = r;
              if (st.rhat_cx) {
                const cx<R> rh = st.rhat_cx[e];
                rr += rh.re * r.re + rh.im * r.im;
                ri += rh.re * r.im - rh.im * r.re;
              } else {
                const R rh = st.rhat[(size_t)i * g.L + l];
                rr += rh * r.re;
                ri += rh * r.im;
              }
              nn += r.re * r.re + r.im * r.im;
            }
            st.x[e] = x;
          }
        }
      }
    }
    const size_t o = (size_t)blockIdx.x * g.K + ct * WAVE;
    wg_store_partial_cx<R>({rr, ri}, p.w, p.lane, valid, st.part_a + o);
    wg_store_partial<R>(nn, p.w, p.lane, valid, st.part_b + o);
  }
}

// Per-column sums of the [G][K] partials, one 256-thread block per 64-column
// tile: wavefront w adds partials w, w + 4, w + 8, ... (independent loads, kept
// in flight by unrolling), then the 4 wavefront sums are added in a fixed
// order.  Every wavefront of the block receives the total.
template <typename T>
__device__ __forceinline__ T block_col_sum(const T* __restrict__ part, int G, int K, int c, bool valid) {
  __shared__ T red[4][WAVE];
  const int w = wave_id(), lane = lane_id();
  T acc = 0;
  if (valid) {
#pragma unroll 8
    for (int b = w; b < G; b += 4) acc += part[(size_t)b * K + c];
  }
  red[w][lane] = acc;
  __syncthreads();
  const T tot = red[0][lane] + red[1][lane] + red[2][lane] + red[3][lane];
  __syncthreads();
  return tot;
}

template <typename R>
__device__ __forceinline__ cx<R> block_col_sum_cx(const cx<R>* part, int G, int K, int c, bool valid) {
  const R* p = reinterpret_cast<const R*>(part);
  // real and imaginary parts are interleaved: sum them as two strided streams
  __shared__ R rr[4][WAVE], ri[4][WAVE];
  const int w = wave_id(), lane = lane_id();
  R ar = 0, ai = 0;
  if (valid) {
#pragma unroll 8
    for (int b = w; b < G; b += 4) {
      const cx<R> v = part[(size_t)b * K + c];
      ar += v.re;
      ai += v.im;
    }
  }
  rr[w][lane] = ar;
  ri[w][lane] = ai;
  __syncthreads();
  const cx<R> tot = {rr[0][lane] + rr[1][lane] + rr[2][lane] + rr[3][lane],
                     ri[0][lane] + ri[1][lane] + ri[2][lane] + ri[3][lane]};
  __syncthreads();
  (void)p;
  return tot;
}

template <typename R>
__device__ __forceinline__ bool cfinite(cx<R> z) { return isfinite(z.re) && isfinite(z.im); }

// The per-column scalar kernels run one block per 64-column tile; wavefront 0
// applies the update after the block-wide reduction.
#define SC_PROLOGUE                              \
  const int c = blockIdx.x * WAVE + lane_id();   \
  const bool valid = c < g.K;                    \
  const bool lead = wave_id() == 0 && valid;

// alpha = rho / (rhat, v)
template <typename R>
__global__ __launch_bounds__(WG) void k_sc_alpha(KGeom g, KrylovState<R> st) {
  SC_PROLOGUE
  const cx<R> rv = block_col_sum_cx(st.part_a, g.G, g.K, c, valid);
  if (!lead || st.flags[c] != COL_ACTIVE) return;
  const cx<R> rho = st.rho[c];
  if ((rv.re == 0 && rv.im == 0) || (rho.re == 0 && rho.im == 0) || !cfinite(rv)) {
    st.flags[c] = COL_BREAKDOWN;
    return;
  }
  st.alpha[c] = cdiv(rho, rv);
  st.iters[c] += 1;
}

// half-step test ||s|| <= tol ||f||
template <typename R>
__global__ __launch_bounds__(WG) void k_sc_half(KGeom g, KrylovState<R> st, R tol) {
  SC_PROLOGUE
  const R sn = sqrt(block_col_sum(st.part_b, g.G, g.K, c, valid));
  if (!lead || st.flags[c] != COL_ACTIVE) return;
  if (sn <= tol * st.fnorm[c]) {
    st.flags[c] = COL_HALF_PENDING;
    st.rnorm[c] = sn;
  }
}

// omega = (t, s) / (t, t)
template <typename R>
__global__ __launch_bounds__(WG) void k_sc_omega(KGeom g, KrylovState<R> st) {
  SC_PROLOGUE
  const cx<R> ts = block_col_sum_cx(st.part_a, g.G, g.K, c, valid);
  const R tt = block_col_sum(st.part_b, g.G, g.K, c, valid);
  if (!lead || st.flags[c] != COL_ACTIVE) return;
  if (tt == 0 || !isfinite(tt)) {
    st.flags[c] = COL_BREAKDOWN;
    return;
  }
  st.omega[c] = {ts.re / tt, ts.im / tt};
}

// rho_new = (rhat, r); ||r|| test; beta = (rho_new / rho)(alpha / omega)
template <typename R>
__global__ __launch_bounds__(WG) void k_sc_beta(KGeom g, KrylovState<R> st, R tol, int maxit) {
  SC_PROLOGUE
  const cx<R> rn = block_col_sum_cx(st.part_a, g.G, g.K, c, valid);
  const R nn = sqrt(block_col_sum(st.part_b, g.G, g.K, c, valid));
  if (!lead) return;
  const int f = st.flags[c];
  if (f == COL_HALF_PENDING) {
    st.flags[c] = COL_HALF_CONVERGED;
    return;
  }
  if (f != COL_ACTIVE) return;
  st.rnorm[c] = nn;
  if (nn <= tol * st.fnorm[c]) {
    st.flags[c] = COL_CONVERGED;
    return;
  }
  if (st.iters[c] >= maxit) {
    st.flags[c] = COL_MAXIT;
    return;
  }
  const cx<R> om = st.omega[c];
  if ((om.re == 0 && om.im == 0) || !cfinite(rn)) {
    st.flags[c] = COL_BREAKDOWN;
    return;
  }
  st.beta[c] = cmul(cdiv(rn, st.rho[c]), cdiv(st.alpha[c], om));
  st.rho[c] = rn;
}

// out = (L U)^{-1} in, one thread per column: forward then backward substitution
// over the rows in order.  The previous row's result stays in a register, so a
// tridiagonal factor has no memory dependence between rows.  Inactive columns
// are skipped (their preconditioned vectors are not used).
template <typename R>
__global__ __launch_bounds__(64) void k_ilu_apply(int n, int K, int L, IluFactors<R> fac, const int* __restrict__ flags,
                                                 const cx<R>* __restrict__ in, cx<R>* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= K || flags[c] != COL_ACTIVE) return;
  const cx<R>* f = fac.f + (size_t)(c / L) * fac.nnz;
  cx<R> prev = {0, 0};
  for (int i = 0; i < n; ++i) {
    cx<R> y = in[(size_t)i * K + c];
    const int kd = fac.diagpos[i];
    for (int k = fac.rowptr[i]; k < kd; ++k) {
      const int j = fac.col[k];
      const cx<R> yj = (j == i - 1) ? prev : out[(size_t)j * K + c];
      y = csub(y, cmul(f[k], yj));
    }
    out[(size_t)i * K + c] = y;
    prev = y;
  }
  prev = {0, 0};
  for (int i = n - 1; i >= 0; --i) {
    cx<R> z = out[(size_t)i * K + c];
    const int kd = fac.diagpos[i];
    for (int k = kd + 1; k < fac.rowptr[i + 1]; ++k) {
      const int j = fac.col[k];
      const cx<R> zj = (j == i + 1) ? prev : out[(size_t)j * K + c];
      z = csub(z, cmul(f[k], zj));
    }
    z = cmul(z, f[kd]);
    out[(size_t)i * K + c] = z;
    prev = z;
  }
}

int* LaunchTimer::begin(hipStream_t s, int kind, double tile_bytes, double fixed) {
  if (used >= capacity || used >= 512) return nullptr;
  recs[used] = {kind, tile_bytes, fixed};
  (void)hipEventRecord(events[2 * used], s);
  return d_counts + used;
}
void LaunchTimer::end(hipStream_t s) {
  (void)hipEventRecord(events[2 * used + 1], s);
  ++used;
}

template <typename R>
void launch_iteration(hipStream_t s, const KGeom& g, const KrylovState<R>& st, const int* rowptr,
                      const int* col, const ab_pair<R>* ab, R tol, int maxit, bool first,
                      const IluFactors<R>* ilu, LaunchTimer* tm, double matrix_bytes) {
  const dim3 grid((unsigned)g.G), blk(WG);
  const dim3 cgrid((unsigned)g.nct), cblk(WG);
  const dim3 igrid((g.K + 63) / 64), iblk(64);
  // algorithmic traffic: n x K complex passes per fully processed launch, plus
  // per-launch fixed bytes (merged CSR; shared real rhat (n, L); diagonals (n, N))
  const double blk_b = (double)g.n * g.K * 2 * sizeof(R);
  const double rhat_b = (double)g.n * g.L * sizeof(R), diag_b = (double)g.n * g.N * 2 * sizeof(R);
  const bool jac = st.p == nullptr;
  int* c;
  // p update: read r (p, v), write p_hat or p; Jacobi reads d and 1/d
  c = tm ? tm->begin(s, 1, (first ? 2 : 4) * blk_b + (jac ? 2 * diag_b : 0), 0) : nullptr;
  k_update_p<R><<<grid, blk, 0, s>>>(g, st, first ? 1 : 0, c);
  if (c) tm->end(s);
  if (ilu) k_ilu_apply<R><<<igrid, iblk, 0, s>>>(g.n, g.K, g.L, *ilu, st.flags, st.p, st.ph);
  // v = S p_hat: gather p_hat once, write v, read rhat; the merged CSR once per launch
  c = tm ? tm->begin(s, 0, 2 * blk_b + rhat_b, matrix_bytes) : nullptr;
  k_spmm_v<R><<<grid, blk, 0, s>>>(g, st, rowptr, col, ab, c);
  if (c) tm->end(s);
  k_sc_alpha<R><<<cgrid, cblk, 0, s>>>(g, st);
  c = tm ? tm->begin(s, 1, 3 * blk_b + (jac ? diag_b : 0), 0) : nullptr;
  k_update_s<R><<<grid, blk, 0, s>>>(g, st, c);
  if (c) tm->end(s);
  k_sc_half<R><<<cgrid, cblk, 0, s>>>(g, st, tol);
  if (ilu) k_ilu_apply<R><<<igrid, iblk, 0, s>>>(g.n, g.K, g.L, *ilu, st.flags, st.s, st.sh);
  c = tm ? tm->begin(s, 0, (jac ? 2 : 3) * blk_b + (jac ? diag_b : 0), matrix_bytes) : nullptr;
  k_spmm_t<R><<<grid, blk, 0, s>>>(g, st, rowptr, col, ab, c);
  if (c) tm->end(s);
  k_sc_omega<R><<<cgrid, cblk, 0, s>>>(g, st);
  c = tm ? tm->begin(s, 1, (first ? 5 : 6) * blk_b + (jac ? 0 : blk_b) + rhat_b + (jac ? diag_b : 0), 0)
         : nullptr;
  k_update_x<R><<<grid, blk, 0, s>>>(g, st, first ? 1 : 0, c);
  if (c) tm->end(s);
  k_sc_beta<R><<<cgrid, cblk, 0, s>>>(g, st, tol, maxit);
}

// x = 0, r = f (broadcast over poles); partials of (rhat, r) = ||f||^2
template <typename R>
__global__ __launch_bounds__(WG) void k_init(KGeom g, KrylovState<R> st, const R* __restrict__ F) {
  const WgPos p = wg_pos(g);
  for (int ct = 0; ct < g.nct; ++ct) {
    const int c = ct * WAVE + p.lane;
    const bool valid = c < g.K;
    R nn = 0;
    if (valid) {
      const int l = c % g.L;
      for (int t = 0; t < g.steps; ++t) {
        const int rb = step_block(g, p, t);
        if (rb < 0) break;
        const int r1 = min((rb + 1) * g.rows_per_block, g.n);
        for (int i = rb * g.rows_per_block + p.w; i < r1; i += 4) {
          const R f = F[(size_t)i * g.L + l];
          st.r[(size_t)i * g.K + c] = {f, 0};
          st.x[(size_t)i * g.K + c] = {0, 0};
          nn += f * f;
        }
      }
    }
    wg_store_partial<R>(nn, p.w, p.lane, valid, st.part_b + (size_t)blockIdx.x * g.K + ct * WAVE);
  }
}

template <typename R>
__global__ __launch_bounds__(WG) void k_init_scalars(KGeom g, KrylovState<R> st) {
  SC_PROLOGUE
  const R nn = block_col_sum(st.part_b, g.G, g.K, c, valid);
  if (!lead) return;
  st.fnorm[c] = sqrt(nn);
  st.rnorm[c] = sqrt(nn);
  st.rho[c] = {nn, 0};
  st.alpha[c] = {1, 0};
  st.omega[c] = {1, 0};
  st.beta[c] = {0, 0};
  st.iters[c] = 0;
  st.flags[c] = nn == 0 ? COL_CONVERGED : COL_ACTIVE;
}

template <typename R>
void launch_init(hipStream_t s, const KGeom& g, const KrylovState<R>& st, const R* F) {
  k_init<R><<<dim3((unsigned)g.G), dim3(WG), 0, s>>>(g, st, F);
}
template <typename R>
void launch_init_scalars(hipStream_t s, const KGeom& g, const KrylovState<R>& st) {
  k_init_scalars<R><<<dim3((unsigned)g.nct), dim3(WG), 0, s>>>(g, st);
}

// ---------------------------------------------------------------------------
// Mixed precision: FP64 defect R = F - S Y and the FP32 <-> FP64 transfers.
__global__ __launch_bounds__(WG) void k_defect(KGeom g, const int* __restrict__ rowptr, const int* __restrict__ col,
                                              const ab_pair<double>* __restrict__ ab,
                                              const cx<double>* __restrict__ sigma_col, const double* __restrict__ F,
                                              const cx<double>* __restrict__ Y, cx<double>* __restrict__ Rout,
                                              double* __restrict__ part) {
  const WgPos p = wg_pos(g);
  for (int ct = 0; ct < g.nct; ++ct) {
    const int c = ct * WAVE + p.lane;
    const bool valid = c < g.K;
    const int cc = min(c, g.K - 1);
    const int l = cc % g.L;
    const cx<double> sig = sigma_col[cc];
    double nn = 0;
    for (int t = 0; t < g.steps; ++t) {
      const int rb = step_block(g, p, t);
      if (rb < 0) break;
      const int r1 = min((rb + 1) * g.rows_per_block, g.n);
      for (int pos = rb * g.rows_per_block + p.w; pos < r1; pos += 4) {
        const int i = g.sched ? g.sched[pos] : pos;
        const double f = F[(size_t)i * g.L + l];
        cx<double> r = {f, 0.0};
        if (Y) {
          const cx<double> q = shifted_row<double, kChunk>(i, rowptr, col, ab, Y + cc, g.K, sig);
          r = {f - q.re, -q.im};
          if (valid) Rout[(size_t)i * g.K + c] = r;
        }
        nn += r.re * r.re + r.im * r.im;
      }
    }
    wg_store_partial<double>(nn, p.w, p.lane, valid, part + (size_t)blockIdx.x * g.K + ct * WAVE);
  }
}

void launch_defect(hipStream_t s, const KGeom& g, const int* rowptr, const int* col, const ab_pair<double>* ab,
                   const cx<double>* sigma_col, const double* F, const cx<double>* Y, cx<double>* Rout,
                   double* part) {
  k_defect<<<dim3((unsigned)g.G), dim3(WG), 0, s>>>(g, rowptr, col, ab, sigma_col, F, Y, Rout, part);
}

__global__ __launch_bounds__(WG) void k_defect_norms(KGeom g, const double* __restrict__ part, double tol, int first,
                                                    double* __restrict__ fnorm, double* __restrict__ scale,
                                                    double* __restrict__ relres) {
  SC_PROLOGUE
  const double r = sqrt(block_col_sum(part, g.G, g.K, c, valid));
  if (!lead) return;
  if (first) fnorm[c] = r;
  const double fn = fnorm[c];
  const bool done = r <= tol * fn;
  scale[c] = done ? 0.0 : r;
  relres[c] = fn > 0 ? r / fn : 0.0;
}

__global__ void k_count_positive(int K, const double* __restrict__ v, int* __restrict__ out) {
  __shared__ int cnt[256];
  int mine = 0;
  for (int c = threadIdx.x; c < K; c += 256) mine += v[c] > 0 ? 1 : 0;
  cnt[threadIdx.x] = mine;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) cnt[threadIdx.x] += cnt[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = cnt[0];
}

void launch_defect_norms(hipStream_t s, const KGeom& g, const double* part, double tol, int first, double* fnorm,
                         double* scale, double* relres, int* count) {
  k_defect_norms<<<dim3((unsigned)g.nct), dim3(WG), 0, s>>>(g, part, tol, first, fnorm, scale, relres);
  k_count_positive<<<1, 256, 0, s>>>(g.K, scale, count);
}

__global__ __launch_bounds__(WG) void k_mixed_rhs(KGeom g, const cx<double>* __restrict__ R,
                                                 const double* __restrict__ F, const double* __restrict__ scale,
                                                 KrylovState<float> st, cx<float>* __restrict__ rhat) {
  const WgPos p = wg_pos(g);
  for (int ct = 0; ct < g.nct; ++ct) {
    const int c = ct * WAVE + p.lane;
    const bool valid = c < g.K;
    float nn = 0;
    if (valid) {
      const double sc = scale[c];
      const double inv = sc > 0 ? 1.0 / sc : 0.0;
      const int l = c % g.L;
      for (int t = 0; t < g.steps; ++t) {
        const int rb = step_block(g, p, t);
        if (rb < 0) break;
        const int r1 = min((rb + 1) * g.rows_per_block, g.n);
        for (int i = rb * g.rows_per_block + p.w; i < r1; i += 4) {
          const size_t e = (size_t)i * g.K + c;
          cx<double> v = R ? R[e] : cx<double>{F[(size_t)i * g.L + l], 0.0};
          const cx<float> r = {(float)(v.re * inv), (float)(v.im * inv)};
          st.r[e] = r;
          rhat[e] = r;
          st.x[e] = {0.f, 0.f};
          nn += r.re * r.re + r.im * r.im;
        }
      }
    }
    wg_store_partial<float>(nn, p.w, p.lane, valid, st.part_b + (size_t)blockIdx.x * g.K + ct * WAVE);
  }
}

void launch_mixed_rhs(hipStream_t s, const KGeom& g, const cx<double>* R, const double* F, const double* scale,
                      const KrylovState<float>& st, cx<float>* rhat) {
  k_mixed_rhs<<<dim3((unsigned)g.G), dim3(WG), 0, s>>>(g, R, F, scale, st, rhat);
}

__global__ void k_accumulate(int64_t total, int K, const cx<float>* __restrict__ x, const double* __restrict__ scale,
                             cx<double>* __restrict__ Y, int first) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const double sc = scale[e % K];
  const cx<float> v = x[e];
  cx<double> y = first ? cx<double>{0.0, 0.0} : Y[e];
  y.re += sc * (double)v.re;
  y.im += sc * (double)v.im;
  Y[e] = y;
}

void launch_accumulate(hipStream_t s, const KGeom& g, const cx<float>* x, const double* scale, cx<double>* Y,
                       int first) {
  const int64_t tot = (int64_t)g.n * g.K;
  k_accumulate<<<dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s>>>(tot, g.K, x, scale, Y, first);
}

__global__ void k_count_active(int K, const int* flags, int* out) {
  __shared__ int cnt[256];
  int c0 = 0;
  for (int c = threadIdx.x; c < K; c += 256) c0 += (flags[c] == COL_ACTIVE) ? 1 : 0;
  cnt[threadIdx.x] = c0;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) cnt[threadIdx.x] += cnt[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = cnt[0];
}
void launch_count_active(hipStream_t s, int K, const int* flags, int* out) {
  k_count_active<<<1, 256, 0, s>>>(K, flags, out);
}

// d = diag(A) - sigma_j diag(B), dinv = 1 / d
template <typename R>
__global__ void k_jacobi(int n, int N, const R* dA, const R* dB, const cx<R>* sigma, cx<R>* d,
                         cx<R>* dinv) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * N) return;
  const int i = (int)(e / N), j = (int)(e % N);
  const cx<R> s = sigma[j];
  const cx<R> v = {dA[i] - s.re * dB[i], -s.im * dB[i]};
  d[e] = v;
  dinv[e] = cdiv(cx<R>{1, 0}, v);
}
template <typename R>
void launch_jacobi_diag(hipStream_t s, int n, int N, const R* diagA, const R* diagB,
                        const cx<R>* sigma, cx<R>* d, cx<R>* dinv) {
  const int64_t tot = (int64_t)n * N;
  k_jacobi<R><<<dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s>>>(n, N, diagA, diagB, sigma, d, dinv);
}

// U[i, l] (+)= sum_j 2 Re(w_j x[i, j L + l])
template <typename R>
__global__ void k_filter_sum(int n, int L, int N, const cx<R>* __restrict__ x, const double* __restrict__ w,
                             double* __restrict__ U, int accumulate) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * L) return;
  const int64_t i = e / L;
  const int l = (int)(e % L);
  const int64_t K = (int64_t)N * L;
  double s = accumulate ? U[e] : 0.0;
  for (int j = 0; j < N; ++j) {
    const cx<R> y = x[i * K + (int64_t)j * L + l];
    s += 2.0 * (w[2 * j] * (double)y.re - w[2 * j + 1] * (double)y.im);
  }
  U[e] = s;
}
template <typename R>
void launch_filter_sum(hipStream_t s, int n, int L, int N, const cx<R>* x, const double* w, double* U,
                       bool accumulate) {
  const int64_t tot = (int64_t)n * L;
  k_filter_sum<R><<<dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s>>>(n, L, N, x, w, U, accumulate ? 1 : 0);
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

// Partial Gram matrices over a chunk of rows: GA = U^T WA, GB = U^T WB.
// A workgroup covers a 128 (rows of G) x 64 (columns of G) region; wavefront w
// covers 64 x 32 of it as 4 x 2 tiles of 16 x 16, for both products.
__global__ __launch_bounds__(WG) void k_gram(int n, int L, const double* __restrict__ U,
                                            const double* __restrict__ WA, const double* __restrict__ WB,
                                            int rows_per_chunk, double* __restrict__ part) {
  const int chunk = blockIdx.x;
  const int nbb = (L + 63) / 64;
  const int ba = blockIdx.y / nbb, bb = blockIdx.y % nbb;
  const int w = wave_id(), lane = lane_id();
  const int a0 = ba * 128 + (w >> 1) * 64;
  const int b0 = bb * 64 + (w & 1) * 32;
  const int li = lane >> 4, lj = lane & 15;
  d4 accA[4][2], accB[4][2];
#pragma unroll
  for (int ta = 0; ta < 4; ++ta)
#pragma unroll
    for (int tb = 0; tb < 2; ++tb) {
      accA[ta][tb] = d4{0, 0, 0, 0};
      accB[ta][tb] = d4{0, 0, 0, 0};
    }
  const int i0 = chunk * rows_per_chunk;
  const int i1 = min(n, i0 + rows_per_chunk);
  for (int i = i0; i < i1; i += 4) {
    const int row = i + li;
    const bool rv = row < i1;
    double a[4], xa[2], xb[2];
#pragma unroll
    for (int ta = 0; ta < 4; ++ta) {
      const int cidx = a0 + 16 * ta + lj;
      a[ta] = (rv && cidx < L) ? U[(size_t)row * L + cidx] : 0.0;
    }
#pragma unroll
    for (int tb = 0; tb < 2; ++tb) {
      const int cidx = b0 + 16 * tb + lj;
      const bool ok = rv && cidx < L;
      xa[tb] = ok ? WA[(size_t)row * L + cidx] : 0.0;
      xb[tb] = ok ? WB[(size_t)row * L + cidx] : 0.0;
    }
#pragma unroll
    for (int ta = 0; ta < 4; ++ta)
#pragma unroll
      for (int tb = 0; tb < 2; ++tb) {
        accA[ta][tb] = mfma64(a[ta], xa[tb], accA[ta][tb]);
        accB[ta][tb] = mfma64(a[ta], xb[tb], accB[ta][tb]);
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
        const int ga = a0 + 16 * ta + li + 4 * q;
        const int gb = b0 + 16 * tb + lj;
        if (ga < L && gb < L) {
          pA[(size_t)ga * L + gb] = accA[ta][tb][q];
          pB[(size_t)ga * L + gb] = accB[ta][tb][q];
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
                 double* part, int nchunks, double* GA, double* GB) {
  int rows = (n + nchunks - 1) / nchunks;
  rows = (rows + 3) / 4 * 4;
  const int tiles = ((L + 127) / 128) * ((L + 63) / 64);
  k_gram<<<dim3(nchunks, tiles), dim3(WG), 0, s>>>(n, L, U, WA, WB, rows, part);
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
  const double* __restrict__ X = gb.X[blockIdx.y];
  double* __restrict__ Y = gb.Y[blockIdx.y];
  const int w = wave_id(), lane = lane_id();
  const int li = lane >> 4, lj = lane & 15;
  const int row0 = blockIdx.x * 64 + w * 16;
  if (row0 >= n) return;
  for (int c0 = 0; c0 < r; c0 += 128) {
    d4 acc[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) acc[t] = d4{0, 0, 0, 0};
    for (int k0 = 0; k0 < L; k0 += 4) {
      const int row = row0 + lj;
      const int k = k0 + li;
      const double a = (row < n && k < L) ? X[(size_t)row * L + k] : 0.0;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int cc = c0 + 16 * t + lj;
        const double b = (k < L && cc < r) ? Z[(size_t)k * r + cc] : 0.0;
        acc[t] = mfma64(a, b, acc[t]);
      }
    }
#pragma unroll
    for (int t = 0; t < 8; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = row0 + li + 4 * q;
        const int cc = c0 + 16 * t + lj;
        if (row < n && cc < r) Y[(size_t)row * r + cc] = acc[t][q];
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
                                      cx<R>*);                                                              \
  template void launch_init<R>(hipStream_t, const KGeom&, const KrylovState<R>&, const R*);                \
  template void launch_init_scalars<R>(hipStream_t, const KGeom&, const KrylovState<R>&);                  \
  template void launch_iteration<R>(hipStream_t, const KGeom&, const KrylovState<R>&, const int*,          \
                                    const int*, const ab_pair<R>*, R, int, bool, const IluFactors<R>*,     \
                                    LaunchTimer*, double);                                                 \
  template void launch_filter_sum<R>(hipStream_t, int, int, int, const cx<R>*, const double*, double*,     \
                                     bool);                                                                 \
  template void launch_spmm_real<R>(hipStream_t, int, int, const int*, const int*, const ab_pair<R>*,      \
                                    const double*, double*, double*);
SLRF_INST(double)
SLRF_INST(float)

}  // namespace slrf

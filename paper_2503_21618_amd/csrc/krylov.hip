// Batched complex-shifted BiCGStab kernels (gfx950).
//
// One launch serves every pole x column of every pencil of a batch.  The
// columns of the batch form a list of 64-column tiles, each tagged with its
// pencil (Batch::tile_inst); the per-pencil sizes, block offsets and CSR
// pointers live in a small device table (Inst).
//
// Work decomposition: a grid of G workgroups of 256 threads (4 wavefronts of
// 64) walks the tiles in order.  Within a tile each lane owns one column and
// each wavefront walks every 4th row of its row blocks, so per-column dot
// products accumulate in registers with no cross-lane traffic.  Workgroup b runs
// on XCD b % 8 (round-robin dispatch).  XCD x owns the contiguous slab of row
// blocks [x * slab, (x + 1) * slab) of the pencil, and its G / 8 workgroups
// advance through the slab together (step t covers x * slab + t * G/8 + [0, G/8)),
// so the rows in flight on one XCD stay close and the neighbours gathered by
// the sparse product are re-read from that XCD's L2.  The 4 wavefronts are
// combined through LDS and the G workgroups by per-column kernels that sum the
// [G][Ktot] partials in a fixed order (bitwise reproducible).
#include "device_util.h"

namespace slrf {

struct WgPos {
  int x, q, per, lane, w;
};

__device__ __forceinline__ WgPos wg_pos(int G) {
  WgPos p;
  p.x = blockIdx.x & 7;
  p.q = blockIdx.x >> 3;
  p.per = G >> 3;
  p.lane = lane_id();
  p.w = wave_id();
  return p;
}

// row block of step t for this workgroup in pencil I, or -1 once past its slab
__device__ __forceinline__ int step_block(const Inst& I, const WgPos& p, int t) {
  const int j = t * p.per + p.q;
  if (j >= I.slab) return -1;
  const int rb = p.x * I.slab + j;
  return rb < I.nrb ? rb : -1;
}

// true if any column of the tile is in one of the given states
__device__ __forceinline__ bool tile_has(const int* flags, int cg, bool valid, int s0, int s1) {
  const int f = valid ? flags[cg] : -1;
  return __any(f == s0 || f == s1);
}

// one vector atomic per processed (workgroup, tile) when instrumented
__device__ __forceinline__ void count_tile(int* counter) {
  if (counter && threadIdx.x == 0) atomicAdd(counter, 1);
}

// Sum of the 4 wavefronts' per-lane values in a fixed order; lane l of wave 0
// stores it at out[l] (out points at this workgroup's slice of the tile).
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

// Complex-shifted sparse product of one row over the merged CSR:
//   q = sum_j (a_ij - sigma b_ij) P[j]      (A - sigma B is never formed)
// The row's entries are taken in chunks of CH.  A chunk's CH column indices and
// (a, b) pairs are contiguous, wave-uniform reads (wide scalar loads; the CSR
// arrays carry kCsrPad zero entries at the end so a chunk never leaves them),
// then CH gathers are issued back to back, then the FMAs.  Entries past the row
// end get zero coefficients and re-read the row's own column; lanes past K read
// a clamped column (both stay in bounds; their contributions are discarded).
template <typename R, int CH>
__device__ __forceinline__ cx<R> shifted_row(int i, cptr<int> rowptr, cptr<int> col, cptr<ab_pair<R>> ab,
                                             const cx<R>* __restrict__ Pc, int K, cx<R> sig) {
  static_assert(CH <= kCsrPad, "chunk longer than the CSR padding");
  const int k0 = rowptr[i], k1 = rowptr[i + 1];
  R apr = 0, api = 0, bpr = 0, bpi = 0;
  for (int kb = k0; kb < k1; kb += CH) {
    int jj[CH];
    ab_pair<R> m[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      jj[u] = col[kb + u];
      m[u] = ldc(ab + kb + u);
    }
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      if (kb + u >= k1) {
        jj[u] = i;
        m[u] = ab_pair<R>{0, 0};
      }
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

// Loop header shared by the batched kernels: tile tg of pencil I; cl is the
// lane's column within the pencil, cc that column clamped into range, cg the
// global column.  FOR_TILES walks every tile; FOR_ACTIVE_TILES walks the list of
// tiles that had an active column at the last poll (the iteration kernels).
#define FOR_TILE_LIST(b, p, COUNT, TG)                                \
  for (int ti_ = 0; ti_ < (COUNT); ++ti_) {                           \
    const int tg = (TG);                                              \
    const Inst I = ldc(as_const((b).inst) + as_const((b).tile_inst)[tg]); \
    const int cl = (tg - I.tile0) * WAVE + (p).lane;                  \
    const bool valid = cl < I.K;                                      \
    const int cc = min(cl, I.K - 1);                                  \
    const int cg = I.col0 + cc;                                       \
    const size_t po = (size_t)blockIdx.x * (b).Ktot + I.col0 + (size_t)(tg - I.tile0) * WAVE;

#define FOR_TILES(b, p) FOR_TILE_LIST(b, p, (b).n_tiles, ti_)
#define FOR_ACTIVE_TILES(b, p) \
  FOR_TILE_LIST(b, p, as_const((const int*)(b).n_active)[0], as_const((const int*)(b).active)[ti_])

#define FOR_ROWS(b, p, I)                                               \
  for (int t_ = 0; t_ < (I).steps; ++t_) {                              \
    const int rb_ = step_block((I), (p), t_);                           \
    if (rb_ < 0) break;                                                 \
    const int r1_ = min((rb_ + 1) * (b).rows_per_block, (I).n);         \
    for (int pos = rb_ * (b).rows_per_block + (p).w; pos < r1_; pos += 4) {

#define END_ROWS \
  }              \
  }

// v = S p_hat, partial (rhat, v)
template <typename R>
__global__ __launch_bounds__(WG) void k_spmm_v(Batch b, KrylovState<R> st, int* counter) {
  const WgPos p = wg_pos(b.G);
  FOR_ACTIVE_TILES(b, p)
    R dr = 0, di = 0;
    if (tile_has(st.flags, cg, valid, COL_ACTIVE, COL_ACTIVE)) {
      count_tile(counter);
      const cx<R> sig = st.sigma_col[cg];
      const int l = cc % I.L;
      const ab_pair<R>* ab = static_cast<const ab_pair<R>*>(I.ab);
      FOR_ROWS(b, p, I)
        const int i = I.sched ? as_const(I.sched)[pos] : pos;
        const size_t e = I.blk + (size_t)i * I.K + cc;
        const cx<R> q = shifted_row<R, kChunk>(i, as_const(I.rowptr), as_const(I.col), as_const(ab),
                                               st.ph + I.blk + cc, I.K, sig);
        if (valid) {
          st.v[e] = q;
          if (st.rhat_cx) {  // conj(rhat) * v
            const cx<R> rh = st.rhat_cx[e];
            dr += rh.re * q.re + rh.im * q.im;
            di += rh.re * q.im - rh.im * q.re;
          } else {
            const R rh = st.rhat[I.rl + (size_t)i * I.L + l];
            dr += rh * q.re;
            di += rh * q.im;
          }
        }
      END_ROWS
    }
    wg_store_partial_cx<R>({dr, di}, p.w, p.lane, valid, st.part_a + po);
  }
}

// t = S s_hat, partials (t, s) = t^H s and (t, t)
template <typename R>
__global__ __launch_bounds__(WG) void k_spmm_t(Batch b, KrylovState<R> st, int* counter) {
  const WgPos p = wg_pos(b.G);
  FOR_ACTIVE_TILES(b, p)
    R tsr = 0, tsi = 0, tt = 0;
    if (tile_has(st.flags, cg, valid, COL_ACTIVE, COL_ACTIVE)) {
      count_tile(counter);
      const cx<R> sig = st.sigma_col[cg];
      const int pole = cc / I.L;
      const ab_pair<R>* ab = static_cast<const ab_pair<R>*>(I.ab);
      FOR_ROWS(b, p, I)
        const int i = I.sched ? as_const(I.sched)[pos] : pos;
        const cx<R> tv = shifted_row<R, kChunk>(i, as_const(I.rowptr), as_const(I.col), as_const(ab),
                                                st.sh + I.blk + cc, I.K, sig);
        if (valid) {
          const size_t e = I.blk + (size_t)i * I.K + cc;
          st.t[e] = tv;
          const cx<R> s = st.s ? st.s[e] : cmul(st.d[I.dn + (size_t)i * I.N + pole], st.sh[e]);
          tsr += tv.re * s.re + tv.im * s.im;  // conj(t) * s
          tsi += tv.re * s.im - tv.im * s.re;
          tt += tv.re * tv.re + tv.im * tv.im;
        }
      END_ROWS
    }
    wg_store_partial_cx<R>({tsr, tsi}, p.w, p.lane, valid, st.part_a + po);
    wg_store_partial<R>(tt, p.w, p.lane, valid, st.part_b + po);
  }
}

// p = r + beta (p - omega v)  (first iteration: p = r).
// Jacobi batch: p itself is not stored; p_hat = p / d with p = d p_hat.
// Batch with ILU(0) pencils: p is stored; the ILU kernel forms p_hat for those
// pencils, and Jacobi pencils of the same batch form p_hat = p / d here.
template <typename R>
__global__ __launch_bounds__(WG) void k_update_p(Batch b, KrylovState<R> st, int first, int* counter) {
  const WgPos p = wg_pos(b.G);
  FOR_ACTIVE_TILES(b, p)
    (void)po;
    if (!tile_has(st.flags, cg, valid, COL_ACTIVE, COL_ACTIVE)) continue;
    count_tile(counter);
    if (!valid || st.flags[cg] != COL_ACTIVE) continue;
    const int pole = cc / I.L;
    const cx<R> beta = st.beta[cg], omega = st.omega[cg];
    FOR_ROWS(b, p, I)
      const int i = pos;
      const size_t e = I.blk + (size_t)i * I.K + cc;
      cx<R> pn = st.r[e];
      if (st.p) {
        if (!first) pn = cadd(pn, cmul(beta, csub(st.p[e], cmul(omega, st.v[e]))));
        st.p[e] = pn;
        if (!I.ilu) st.ph[e] = cmul(pn, st.dinv[I.dn + (size_t)i * I.N + pole]);
      } else {
        const size_t de = I.dn + (size_t)i * I.N + pole;
        if (!first) pn = cadd(pn, cmul(beta, csub(cmul(st.d[de], st.ph[e]), cmul(omega, st.v[e]))));
        st.ph[e] = cmul(pn, st.dinv[de]);
      }
    END_ROWS
  }
}

// s = r - alpha v (Jacobi batch: s_hat = s / d is stored instead; in a batch
// with ILU(0) pencils s is stored, plus s_hat = s / d for its Jacobi pencils) ;
// partial |s|^2
template <typename R>
__global__ __launch_bounds__(WG) void k_update_s(Batch b, KrylovState<R> st, int* counter) {
  const WgPos p = wg_pos(b.G);
  FOR_ACTIVE_TILES(b, p)
    R ss = 0;
    if (tile_has(st.flags, cg, valid, COL_ACTIVE, COL_ACTIVE)) {
      count_tile(counter);
      if (valid && st.flags[cg] == COL_ACTIVE) {
        const int pole = cc / I.L;
        const cx<R> alpha = st.alpha[cg];
        FOR_ROWS(b, p, I)
          const int i = pos;
          const size_t e = I.blk + (size_t)i * I.K + cc;
          const cx<R> s = csub(st.r[e], cmul(alpha, st.v[e]));
          ss += s.re * s.re + s.im * s.im;
          if (st.s) st.s[e] = s;
          if (!st.s || !I.ilu) st.sh[e] = cmul(s, st.dinv[I.dn + (size_t)i * I.N + pole]);
        END_ROWS
      }
    }
    wg_store_partial<R>(ss, p.w, p.lane, valid, st.part_b + po);
  }
}

// x += alpha p_hat + omega s_hat ; r = s - omega t ; partials (rhat, r), |r|^2
// Columns that converged at the half step take x += alpha p_hat only.
template <typename R>
__global__ __launch_bounds__(WG) void k_update_x(Batch b, KrylovState<R> st, int first, int* counter) {
  const WgPos p = wg_pos(b.G);
  FOR_ACTIVE_TILES(b, p)
    R rr = 0, ri = 0, nn = 0;
    if (tile_has(st.flags, cg, valid, COL_ACTIVE, COL_HALF_PENDING)) {
      count_tile(counter);
      const int f = valid ? st.flags[cg] : -1;
      const bool act = f == COL_ACTIVE, half = f == COL_HALF_PENDING;
      if (act || half) {
        const int pole = cc / I.L;
        const int l = cc % I.L;
        const cx<R> alpha = st.alpha[cg];
        const cx<R> omega = act ? st.omega[cg] : cx<R>{0, 0};
        FOR_ROWS(b, p, I)
          const int i = pos;
          const size_t e = I.blk + (size_t)i * I.K + cc;
          cx<R> x = first ? cx<R>{0, 0} : st.x[e];
          x = cadd(x, cmul(alpha, st.ph[e]));
          if (act) {
            const cx<R> sh = st.sh[e];
            x = cadd(x, cmul(omega, sh));
            const cx<R> sv = st.s ? st.s[e] : cmul(st.d[I.dn + (size_t)i * I.N + pole], sh);
            const cx<R> r = csub(sv, cmul(omega, st.t[e]));
            st.r[e] = r;
            if (st.rhat_cx) {
              const cx<R> rh = st.rhat_cx[e];
              rr += rh.re * r.re + rh.im * r.im;
              ri += rh.re * r.im - rh.im * r.re;
            } else {
              const R rh = st.rhat[I.rl + (size_t)i * I.L + l];
              rr += rh * r.re;
              ri += rh * r.im;
            }
            nn += r.re * r.re + r.im * r.im;
          }
          st.x[e] = x;
        END_ROWS
      }
    }
    wg_store_partial_cx<R>({rr, ri}, p.w, p.lane, valid, st.part_a + po);
    wg_store_partial<R>(nn, p.w, p.lane, valid, st.part_b + po);
  }
}

// x = 0, r = f (broadcast over poles); partials of ||f||^2
template <typename R>
__global__ __launch_bounds__(WG) void k_init(Batch b, KrylovState<R> st, const R* __restrict__ F) {
  const WgPos p = wg_pos(b.G);
  FOR_TILES(b, p)
    R nn = 0;
    if (valid) {
      const int l = cc % I.L;
      FOR_ROWS(b, p, I)
        const int i = pos;
        const R f = F[I.rl + (size_t)i * I.L + l];
        const size_t e = I.blk + (size_t)i * I.K + cc;
        st.r[e] = {f, 0};
        st.x[e] = {0, 0};
        nn += f * f;
      END_ROWS
    }
    wg_store_partial<R>(nn, p.w, p.lane, valid, st.part_b + po);
  }
}

// ---------------------------------------------------------------------------
// Per-column scalar kernels: one 256-thread block per global tile.  The sum
// over the G partials is split across the 4 wavefronts (partials w, w + 4, ...,
// loads kept in flight by unrolling) and combined in a fixed order; wavefront 0
// then applies the update.
template <typename T>
__device__ __forceinline__ T block_col_sum(const T* __restrict__ part, int G, int Ktot, int c, bool valid) {
  __shared__ T red[4][WAVE];
  const int w = wave_id(), lane = lane_id();
  T acc = 0;
  if (valid) {
#pragma unroll 8
    for (int g = w; g < G; g += 4) acc += part[(size_t)g * Ktot + c];
  }
  red[w][lane] = acc;
  __syncthreads();
  const T tot = red[0][lane] + red[1][lane] + red[2][lane] + red[3][lane];
  __syncthreads();
  return tot;
}

template <typename R>
__device__ __forceinline__ cx<R> block_col_sum_cx(const cx<R>* part, int G, int Ktot, int c, bool valid) {
  __shared__ R rr[4][WAVE], ri[4][WAVE];
  const int w = wave_id(), lane = lane_id();
  R ar = 0, ai = 0;
  if (valid) {
#pragma unroll 8
    for (int g = w; g < G; g += 4) {
      const cx<R> v = part[(size_t)g * Ktot + c];
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
  return tot;
}

template <typename R>
__device__ __forceinline__ bool cfinite(cx<R> z) { return isfinite(z.re) && isfinite(z.im); }

#define SC_PROLOGUE                                         \
  const Inst I = ldc(as_const(b.inst) + as_const(b.tile_inst)[blockIdx.x]); \
  const int cl = (blockIdx.x - I.tile0) * WAVE + lane_id(); \
  const bool valid = cl < I.K;                              \
  const int c = I.col0 + min(cl, I.K - 1);                  \
  const bool lead = wave_id() == 0 && valid;

// alpha = rho / (rhat, v)
template <typename R>
__global__ __launch_bounds__(WG) void k_sc_alpha(Batch b, KrylovState<R> st) {
  SC_PROLOGUE
  if (!tile_has(st.flags, c, valid, COL_ACTIVE, COL_ACTIVE)) return;
  const cx<R> rv = block_col_sum_cx(st.part_a, b.G, b.Ktot, c, valid);
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
__global__ __launch_bounds__(WG) void k_sc_half(Batch b, KrylovState<R> st, R tol) {
  SC_PROLOGUE
  if (!tile_has(st.flags, c, valid, COL_ACTIVE, COL_ACTIVE)) return;
  const R sn = sqrt(block_col_sum(st.part_b, b.G, b.Ktot, c, valid));
  if (!lead || st.flags[c] != COL_ACTIVE) return;
  if (sn <= (st.tolc ? st.tolc[c] : tol) * st.fnorm[c]) {
    st.flags[c] = COL_HALF_PENDING;
    st.rnorm[c] = sn;
  }
}

// omega = (t, s) / (t, t)
template <typename R>
__global__ __launch_bounds__(WG) void k_sc_omega(Batch b, KrylovState<R> st) {
  SC_PROLOGUE
  if (!tile_has(st.flags, c, valid, COL_ACTIVE, COL_ACTIVE)) return;
  const cx<R> ts = block_col_sum_cx(st.part_a, b.G, b.Ktot, c, valid);
  const R tt = block_col_sum(st.part_b, b.G, b.Ktot, c, valid);
  if (!lead || st.flags[c] != COL_ACTIVE) return;
  if (tt == 0 || !isfinite(tt)) {
    st.flags[c] = COL_BREAKDOWN;
    return;
  }
  st.omega[c] = {ts.re / tt, ts.im / tt};
}

// rho_new = (rhat, r); ||r|| test; beta = (rho_new / rho)(alpha / omega)
template <typename R>
__global__ __launch_bounds__(WG) void k_sc_beta(Batch b, KrylovState<R> st, R tol, int maxit) {
  SC_PROLOGUE
  if (!tile_has(st.flags, c, valid, COL_ACTIVE, COL_HALF_PENDING)) return;
  const cx<R> rn = block_col_sum_cx(st.part_a, b.G, b.Ktot, c, valid);
  const R nn = sqrt(block_col_sum(st.part_b, b.G, b.Ktot, c, valid));
  if (!lead) return;
  const int f = st.flags[c];
  if (f == COL_HALF_PENDING) {
    st.flags[c] = COL_HALF_CONVERGED;
    return;
  }
  if (f != COL_ACTIVE) return;
  st.rnorm[c] = nn;
  if (nn <= (st.tolc ? st.tolc[c] : tol) * st.fnorm[c]) {
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

template <typename R>
__global__ __launch_bounds__(WG) void k_init_scalars(Batch b, KrylovState<R> st) {
  SC_PROLOGUE
  if (threadIdx.x == 0) {  // every tile starts on the active list
    b.active[blockIdx.x] = blockIdx.x;
    if (blockIdx.x == 0) b.n_active[0] = b.n_tiles;
  }
  const R nn = block_col_sum(st.part_b, b.G, b.Ktot, c, valid);
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

// out = (L U)^{-1} in, one thread per global column: forward then backward
// substitution over the rows in order.  The previous row's result stays in a
// register, so a tridiagonal factor has no memory dependence between rows.
// Inactive columns are skipped (their preconditioned vectors are not used).
template <typename R>
__global__ __launch_bounds__(64) void k_ilu_apply(Batch b, const int* __restrict__ flags,
                                                 const cx<R>* __restrict__ in, cx<R>* __restrict__ out) {
  const int cg = blockIdx.x * blockDim.x + threadIdx.x;
  if (cg >= b.Ktot || flags[cg] != COL_ACTIVE) return;
  const Inst I = b.inst[b.col_inst[cg]];
  if (!I.ilu) return;
  const int c = cg - I.col0;
  const cx<R>* f = static_cast<const cx<R>*>(I.ilu) + (size_t)(c / I.L) * I.nnz;
  const cx<R>* src = in + I.blk + c;
  cx<R>* dst = out + I.blk + c;
  cx<R> prev = {0, 0};
  for (int i = 0; i < I.n; ++i) {
    cx<R> y = src[(size_t)i * I.K];
    const int kd = I.diagpos[i];
    for (int k = I.rowptr[i]; k < kd; ++k) {
      const int j = I.col[k];
      const cx<R> yj = (j == i - 1) ? prev : dst[(size_t)j * I.K];
      y = csub(y, cmul(f[k], yj));
    }
    dst[(size_t)i * I.K] = y;
    prev = y;
  }
  prev = {0, 0};
  for (int i = I.n - 1; i >= 0; --i) {
    cx<R> z = dst[(size_t)i * I.K];
    const int kd = I.diagpos[i];
    for (int k = kd + 1; k < I.rowptr[i + 1]; ++k) {
      const int j = I.col[k];
      const cx<R> zj = (j == i + 1) ? prev : dst[(size_t)j * I.K];
      z = csub(z, cmul(f[k], zj));
    }
    z = cmul(z, f[kd]);
    dst[(size_t)i * I.K] = z;
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
void launch_iteration(hipStream_t s, const Batch& b, const KrylovState<R>& st, R tol, int maxit, bool first,
                      bool ilu, LaunchTimer* tm, const IterBytes& by) {
  const dim3 grid((unsigned)b.G), blk(WG);
  const dim3 cgrid((unsigned)b.n_tiles), cblk(WG);
  const dim3 igrid((unsigned)((b.Ktot + 63) / 64)), iblk(64);
  const bool jac = st.p == nullptr;
  int* c;
  // p update: read r (p, v), write p_hat or p; Jacobi reads d and 1/d
  c = tm ? tm->begin(s, 1, (first ? 2 : 4) * by.blk + (jac ? 2 * by.diag : 0), 0) : nullptr;
  k_update_p<R><<<grid, blk, 0, s>>>(b, st, first ? 1 : 0, c);
  if (c) tm->end(s);
  if (ilu) k_ilu_apply<R><<<igrid, iblk, 0, s>>>(b, st.flags, st.p, st.ph);
  // v = S p_hat: gather p_hat once, write v, read rhat; the merged CSR once per launch
  c = tm ? tm->begin(s, 0, 2 * by.blk + by.rhat, by.matrix) : nullptr;
  k_spmm_v<R><<<grid, blk, 0, s>>>(b, st, c);
  if (c) tm->end(s);
  k_sc_alpha<R><<<cgrid, cblk, 0, s>>>(b, st);
  c = tm ? tm->begin(s, 1, 3 * by.blk + (jac ? by.diag : 0), 0) : nullptr;
  k_update_s<R><<<grid, blk, 0, s>>>(b, st, c);
  if (c) tm->end(s);
  k_sc_half<R><<<cgrid, cblk, 0, s>>>(b, st, tol);
  if (ilu) k_ilu_apply<R><<<igrid, iblk, 0, s>>>(b, st.flags, st.s, st.sh);
  c = tm ? tm->begin(s, 0, (jac ? 2 : 3) * by.blk + (jac ? by.diag : 0), by.matrix) : nullptr;
  k_spmm_t<R><<<grid, blk, 0, s>>>(b, st, c);
  if (c) tm->end(s);
  k_sc_omega<R><<<cgrid, cblk, 0, s>>>(b, st);
  c = tm ? tm->begin(s, 1, (first ? 5 : 6) * by.blk + (jac ? 0 : by.blk) + by.rhat + (jac ? by.diag : 0), 0)
         : nullptr;
  k_update_x<R><<<grid, blk, 0, s>>>(b, st, first ? 1 : 0, c);
  if (c) tm->end(s);
  k_sc_beta<R><<<cgrid, cblk, 0, s>>>(b, st, tol, maxit);
}

template <typename R>
void launch_init(hipStream_t s, const Batch& b, const KrylovState<R>& st, const R* F) {
  k_init<R><<<dim3((unsigned)b.G), dim3(WG), 0, s>>>(b, st, F);
}
template <typename R>
void launch_init_scalars(hipStream_t s, const Batch& b, const KrylovState<R>& st) {
  k_init_scalars<R><<<dim3((unsigned)b.n_tiles), dim3(WG), 0, s>>>(b, st);
}

// Number of active columns, and the ordered list of tiles that still have an
// active column (one block; tiles in chunks of 256 with an LDS prefix sum).
__global__ __launch_bounds__(256) void k_count_active(Batch b, const int* __restrict__ flags,
                                                     int* __restrict__ out) {
  __shared__ int scan[256];
  __shared__ int cols[256];
  int base = 0, ncols = 0;
  for (int t0 = 0; t0 < b.n_tiles; t0 += 256) {
    const int t = t0 + (int)threadIdx.x;
    int act = 0, cnt = 0;
    if (t < b.n_tiles) {
      const Inst I = b.inst[b.tile_inst[t]];
      const int c0 = I.col0 + (t - I.tile0) * WAVE;
      const int c1 = min(c0 + WAVE, I.col0 + I.K);
      for (int c = c0; c < c1; ++c) cnt += flags[c] == COL_ACTIVE ? 1 : 0;
      act = cnt > 0 ? 1 : 0;
    }
    scan[threadIdx.x] = act;
    cols[threadIdx.x] = cnt;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {  // inclusive Hillis-Steele scan
      const int v = threadIdx.x >= (unsigned)off ? scan[threadIdx.x - off] : 0;
      const int w = threadIdx.x >= (unsigned)off ? cols[threadIdx.x - off] : 0;
      __syncthreads();
      scan[threadIdx.x] += v;
      cols[threadIdx.x] += w;
      __syncthreads();
    }
    if (act) b.active[base + scan[threadIdx.x] - 1] = t;
    base += scan[255];
    ncols += cols[255];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    b.n_active[0] = base;
    out[0] = ncols;
  }
}
void launch_count_active(hipStream_t s, const Batch& b, const int* flags, int* out) {
  k_count_active<<<1, 256, 0, s>>>(b, flags, out);
}

// ---------------------------------------------------------------------------
// Mixed precision: FP64 defect R = F - S Y and the FP32 <-> FP64 transfers.
__global__ __launch_bounds__(WG) void k_defect(Batch b, const cx<double>* __restrict__ sigma_col,
                                              const double* __restrict__ F, const cx<double>* __restrict__ Y,
                                              cx<double>* __restrict__ Rout, double* __restrict__ part) {
  const WgPos p = wg_pos(b.G);
  FOR_TILES(b, p)
    const int l = cc % I.L;
    const cx<double> sig = sigma_col[cg];
    double nn = 0;
    FOR_ROWS(b, p, I)
      const int i = I.sched ? as_const(I.sched)[pos] : pos;
      const double f = F[I.rl + (size_t)i * I.L + l];
      cx<double> r = {f, 0.0};
      if (Y) {
        const cx<double> q = shifted_row<double, kChunk>(i, as_const(I.rowptr), as_const(I.col), as_const(I.ab64),
                                                         Y + I.blk + cc, I.K, sig);
        r = {f - q.re, -q.im};
        if (valid) Rout[I.blk + (size_t)i * I.K + cc] = r;
      }
      nn += r.re * r.re + r.im * r.im;
    END_ROWS
    wg_store_partial<double>(nn, p.w, p.lane, valid, part + po);
  }
}

void launch_defect(hipStream_t s, const Batch& b, const cx<double>* sigma_col, const double* F,
                   const cx<double>* Y, cx<double>* Rout, double* part) {
  k_defect<<<dim3((unsigned)b.G), dim3(WG), 0, s>>>(b, sigma_col, F, Y, Rout, part);
}

// scale_c = ||R_c|| unless the defect meets its target; the next FP32 solve of
// the column only has to reduce R_c by the remaining factor target ||F|| / ||R||,
// so its tolerance is a tenth of that, within [min32, 1e-1].
__global__ __launch_bounds__(WG) void k_defect_norms(Batch b, const double* __restrict__ part,
                                                    const double* __restrict__ tol, int first,
                                                    double* __restrict__ fnorm, double* __restrict__ scale,
                                                    double* __restrict__ relres, float* __restrict__ tol32,
                                                    double min32) {
  SC_PROLOGUE
  const double r = sqrt(block_col_sum(part, b.G, b.Ktot, c, valid));
  if (!lead) return;
  if (first) fnorm[c] = r;
  const double fn = fnorm[c];
  const bool done = r <= tol[c] * fn;
  scale[c] = done ? 0.0 : r;
  relres[c] = fn > 0 ? r / fn : 0.0;
  const double gap = r > 0 ? tol[c] * fn / r : 1.0;
  tol32[c] = (float)fmin(1e-1, fmax(min32, 0.1 * gap));
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

void launch_defect_norms(hipStream_t s, const Batch& b, const double* part, const double* tol, int first,
                         double* fnorm, double* scale, double* relres, float* tol32, double min32, int* count) {
  k_defect_norms<<<dim3((unsigned)b.n_tiles), dim3(WG), 0, s>>>(b, part, tol, first, fnorm, scale, relres,
                                                                tol32, min32);
  k_count_positive<<<1, 256, 0, s>>>(b.Ktot, scale, count);
}

__global__ __launch_bounds__(WG) void k_mixed_rhs(Batch b, const cx<double>* __restrict__ R,
                                                 const double* __restrict__ F, const double* __restrict__ scale,
                                                 KrylovState<float> st, cx<float>* __restrict__ rhat) {
  const WgPos p = wg_pos(b.G);
  FOR_TILES(b, p)
    float nn = 0;
    if (valid) {
      const double sc = scale[cg];
      const double inv = sc > 0 ? 1.0 / sc : 0.0;
      const int l = cc % I.L;
      FOR_ROWS(b, p, I)
        const int i = pos;
        const size_t e = I.blk + (size_t)i * I.K + cc;
        const cx<double> v = R ? R[e] : cx<double>{F[I.rl + (size_t)i * I.L + l], 0.0};
        const cx<float> r = {(float)(v.re * inv), (float)(v.im * inv)};
        st.r[e] = r;
        rhat[e] = r;
        st.x[e] = {0.f, 0.f};
        nn += r.re * r.re + r.im * r.im;
      END_ROWS
    }
    wg_store_partial<float>(nn, p.w, p.lane, valid, st.part_b + po);
  }
}

void launch_mixed_rhs(hipStream_t s, const Batch& b, const cx<double>* R, const double* F, const double* scale,
                      const KrylovState<float>& st, cx<float>* rhat) {
  k_mixed_rhs<<<dim3((unsigned)b.G), dim3(WG), 0, s>>>(b, R, F, scale, st, rhat);
}

__global__ __launch_bounds__(WG) void k_accumulate(Batch b, const cx<float>* __restrict__ x,
                                                  const double* __restrict__ scale, cx<double>* __restrict__ Y,
                                                  int first) {
  const WgPos p = wg_pos(b.G);
  FOR_TILES(b, p)
    (void)po;
    if (!valid) continue;
    const double sc = scale[cg];
    FOR_ROWS(b, p, I)
      const size_t e = I.blk + (size_t)pos * I.K + cc;
      const cx<float> v = x[e];
      cx<double> y = first ? cx<double>{0.0, 0.0} : Y[e];
      y.re += sc * (double)v.re;
      y.im += sc * (double)v.im;
      Y[e] = y;
    END_ROWS
  }
}

void launch_accumulate(hipStream_t s, const Batch& b, const cx<float>* x, const double* scale, cx<double>* Y,
                       int first) {
  k_accumulate<<<dim3((unsigned)b.G), dim3(WG), 0, s>>>(b, x, scale, Y, first);
}

#define SLRF_INST(R)                                                                                  \
  template void launch_init<R>(hipStream_t, const Batch&, const KrylovState<R>&, const R*);        \
  template void launch_init_scalars<R>(hipStream_t, const Batch&, const KrylovState<R>&);          \
  template void launch_iteration<R>(hipStream_t, const Batch&, const KrylovState<R>&, R, int, bool, \
                                    bool, LaunchTimer*, const IterBytes&);
SLRF_INST(double)
SLRF_INST(float)

}  // namespace slrf

// Batched complex-shifted BiCGStab kernels (gfx950).
//
// One launch serves every pole x column of every pencil of a batch.  The
// columns of the batch form a list of tiles, each tagged with its pencil
// (Batch::tile_inst); the per-pencil sizes, block offsets and CSR pointers live
// in a small device table (Inst).
//
// Lane width.  A lane owns V adjacent columns: V = 1 for complex FP64 (16 B per
// element), V = 2 for complex FP32, so that every gather and vector access moves
// 16 B per lane in both precisions.  A tile is W = 64 V columns.  A pencil has
// Kp = K rounded up to a multiple of W columns; the padding columns have a zero
// right-hand side and are never active.  Its blocks are stored tile-major: tile
// t is an n x W row-major panel (see tile_base), so each row of a tile is one
// 1 KB line-aligned slice and the panel of a tile is contiguous.
//
// Work decomposition: a grid of G workgroups of 256 threads (4 wavefronts of
// 64) walks the tiles in order.  Within a tile each wavefront walks every 4th
// row of its row blocks, so per-column dot products accumulate in registers with
// no cross-lane traffic.  Workgroup b runs on XCD b % 8 (round-robin dispatch).
// XCD x owns the contiguous slab of row blocks [x * slab, (x + 1) * slab) of the
// pencil, and its G / 8 workgroups advance through the slab together (step t
// covers x * slab + t * G/8 + [0, G/8)), so the rows in flight on one XCD stay
// close and the neighbours gathered by the sparse product are re-read from that
// XCD's L2.  The 4 wavefronts are combined through LDS and the G workgroups by
// per-column kernels that sum the [G][Ktot] partials in a fixed order (bitwise
// reproducible).  A pencil's row-block slots are rotated over the XCD's
// workgroups by Inst::rot, so a batch of small pencils loads them evenly.
#include "device_util.h"

namespace slrf {

template <typename R>
struct LaneWidth {
  static constexpr int V = sizeof(R) == 4 ? 2 : 1;
};

// V adjacent complex values of one row, loaded and stored as one 16 B access.
template <typename R, int V>
struct alignas(V * sizeof(cx<R>)) cvec {
  cx<R> c[V];
};

template <typename R, int V>
__device__ __forceinline__ cvec<R, V> ldv(const cx<R>* p) {
  return *reinterpret_cast<const cvec<R, V>*>(p);
}
template <typename R, int V>
__device__ __forceinline__ void stv(cx<R>* p, const cvec<R, V>& v) {
  *reinterpret_cast<cvec<R, V>*>(p) = v;
}

// Streamed blocks (written or read once per launch): non-temporal accesses, so
// that they do not evict the gathered input rows from L2.
template <typename R, int V>
__device__ __forceinline__ cvec<R, V> ldv_nt(const cx<R>* p) {
  using W = R __attribute__((ext_vector_type(2 * V)));
  const W w = __builtin_nontemporal_load(reinterpret_cast<const W*>(p));
  cvec<R, V> out;
#pragma unroll
  for (int v = 0; v < V; ++v) out.c[v] = {w[2 * v], w[2 * v + 1]};
  return out;
}
template <typename R, int V>
__device__ __forceinline__ void stv_nt(cx<R>* p, const cvec<R, V>& v) {
  using W = R __attribute__((ext_vector_type(2 * V)));
  W w;
#pragma unroll
  for (int u = 0; u < V; ++u) {
    w[2 * u] = v.c[u].re;
    w[2 * u + 1] = v.c[u].im;
  }
  __builtin_nontemporal_store(w, reinterpret_cast<W*>(p));
}

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
  const int j = t * p.per + (p.q + I.rot) % p.per;
  if (j >= I.slab) return -1;
  const int rb = p.x * I.slab + j;
  return rb < I.nrb ? rb : -1;
}

// Flags of the lane's V columns (-1 for columns past K).
template <int V>
__device__ __forceinline__ void lane_flags(const int* flags, int cg0, int cl0, int K, int (&f)[V]) {
#pragma unroll
  for (int v = 0; v < V; ++v) f[v] = cl0 + v < K ? flags[cg0 + v] : -1;
}

// true if any column of the tile is in one of the given states
template <int V>
__device__ __forceinline__ bool tile_has(const int* flags, int cg0, int cl0, int K, int s0, int s1) {
  int f[V];
  lane_flags<V>(flags, cg0, cl0, K, f);
  bool any = false;
#pragma unroll
  for (int v = 0; v < V; ++v) any |= f[v] == s0 || f[v] == s1;
  return __any(any);
}

// one vector atomic per processed (workgroup, tile) when instrumented
__device__ __forceinline__ void count_tile(int* counter) {
  if (counter && threadIdx.x == 0) atomicAdd(counter, 1);
}

// The partial sums of a workgroup that owns no rows of a tile's pencil are
// zero: wavefront 0 stores them directly (the values wg_store_partial would
// store), with no flags, LDS reduction or barrier.  In a batch of small
// pencils most (workgroup, tile) pairs are of this kind.
template <typename T, int V>
__device__ __forceinline__ void zero_partial(int w, int lane, int cl0, int K, T* out) {
  if (w != 0) return;
#pragma unroll
  for (int u = 0; u < V; ++u)
    if (cl0 + u < K) out[V * lane + u] = T(0);
}

template <typename R, int V>
__device__ __forceinline__ void zero_partial_cx(int w, int lane, int cl0, int K, cx<R>* out) {
  if (w != 0) return;
#pragma unroll
  for (int u = 0; u < V; ++u)
    if (cl0 + u < K) out[V * lane + u] = cx<R>{0, 0};
}

// Sums of the 4 wavefronts' per-lane values in a fixed order; lane l of wave 0
// stores column v's sum at out[V l + v] (out points at this workgroup's slice of
// the tile), for the columns before K.
template <typename T, int V>
__device__ __forceinline__ void wg_store_partial(const T (&v)[V], int w, int lane, int cl0, int K, T* out) {
  __shared__ T red[4][V * WAVE];
#pragma unroll
  for (int u = 0; u < V; ++u) red[w][V * lane + u] = v[u];
  __syncthreads();
  if (w == 0) {
#pragma unroll
    for (int u = 0; u < V; ++u) {
      const int k = V * lane + u;
      if (cl0 + u < K) out[k] = red[0][k] + red[1][k] + red[2][k] + red[3][k];
    }
  }
  __syncthreads();
}

template <typename R, int V>
__device__ __forceinline__ void wg_store_partial_cx(const cx<R> (&v)[V], int w, int lane, int cl0, int K,
                                                    cx<R>* out) {
  __shared__ R rr[4][V * WAVE], ri[4][V * WAVE];
#pragma unroll
  for (int u = 0; u < V; ++u) {
    rr[w][V * lane + u] = v[u].re;
    ri[w][V * lane + u] = v[u].im;
  }
  __syncthreads();
  if (w == 0) {
#pragma unroll
    for (int u = 0; u < V; ++u) {
      const int k = V * lane + u;
      if (cl0 + u < K)
        out[k] = {rr[0][k] + rr[1][k] + rr[2][k] + rr[3][k], ri[0][k] + ri[1][k] + ri[2][k] + ri[3][k]};
    }
  }
  __syncthreads();
}

// Complex-shifted sparse product of one row over the merged CSR, for the lane's
// V columns:  q_v = sum_j (a_ij - sigma_v b_ij) P[j][v]   (A - sigma B is never
// formed).  The row's entries are taken in chunks of CH.  A chunk's CH column
// indices and (a, b) pairs are contiguous, wave-uniform reads (wide scalar
// loads; the CSR arrays carry kCsrPad zero entries at the end so a chunk never
// leaves them), then CH gathers of 16 B per lane are issued back to back, then
// the FMAs.  Entries past the row end get zero coefficients and re-read the
// row's own column; lanes past K read a clamped column (both stay in bounds;
// their contributions are discarded).  PZ: the re-read values are replaced by
// zeros as well, for gathers from a vector whose own row may not be written yet
// (a colour sweep), where 0 times leftover bits could be NaN.
template <typename R, int V, int CH, bool PZ = false>
__device__ __forceinline__ cvec<R, V> shifted_row(int i, cptr<int> rowptr, cptr<int> col, cptr<ab_pair<R>> ab,
                                                  const cx<R>* __restrict__ Pc, int ld, const cx<R> (&sig)[V]) {
  static_assert(CH <= kCsrPad, "chunk longer than the CSR padding");
  const int k0 = rowptr[i], k1 = rowptr[i + 1];
  R apr[V] = {}, api[V] = {}, bpr[V] = {}, bpi[V] = {};
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
    cvec<R, V> x[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u) x[u] = ldv<R, V>(Pc + (size_t)jj[u] * ld);
    if constexpr (PZ) {
#pragma unroll
      for (int u = 0; u < CH; ++u)
        if (kb + u >= k1) x[u] = cvec<R, V>{};
    }
#pragma unroll
    for (int u = 0; u < CH; ++u) {
#pragma unroll
      for (int v = 0; v < V; ++v) {
        apr[v] += m[u].a * x[u].c[v].re;
        api[v] += m[u].a * x[u].c[v].im;
        bpr[v] += m[u].b * x[u].c[v].re;
        bpi[v] += m[u].b * x[u].c[v].im;
      }
    }
  }
  cvec<R, V> q;
#pragma unroll
  for (int v = 0; v < V; ++v)
    q.c[v] = {apr[v] - (sig[v].re * bpr[v] - sig[v].im * bpi[v]),
              api[v] - (sig[v].re * bpi[v] + sig[v].im * bpr[v])};
  return q;
}

constexpr int kChunk = 16;
// Chunk of the generic rows inside the shared-gather variants: 8 entries in
// FP32 keeps those kernels within 128 VGPRs (16 spilled registers otherwise).
template <typename R>
constexpr int kChunkShared = sizeof(R) == 4 ? 8 : kChunk;
constexpr int kGroupRows = 4;  // rows of a stencil group (flags built on the host)

// Complex-shifted sparse product of a stencil group: rows i0 .. i0 + 3 whose
// entries have the same offsets col - row, in runs of three consecutive columns
// (checked on the host).  Run j of row r covers columns c_j + r .. c_j + r + 2,
// so the six input rows c_j .. c_j + 5 are gathered once for the four rows:
// 6 gathers per run instead of 12.  Each row's entries are summed in entry
// order, as in shifted_row.
template <typename R, int V>
__device__ __forceinline__ void shifted_group(int i0, cptr<int> rowptr, cptr<int> col, cptr<ab_pair<R>> ab,
                                              const cx<R>* __restrict__ Pc, int ld, const cx<R> (&sig)[V],
                                              cvec<R, V> (&q)[kGroupRows]) {
  int kb[kGroupRows];
#pragma unroll
  for (int r = 0; r < kGroupRows; ++r) kb[r] = rowptr[i0 + r];
  const int m = rowptr[i0 + 1] - kb[0];
  R apr[kGroupRows][V] = {}, api[kGroupRows][V] = {}, bpr[kGroupRows][V] = {}, bpi[kGroupRows][V] = {};
#pragma unroll 1
  for (int j = 0; j < m; j += 3) {
    const int c0 = col[kb[0] + j];
    cvec<R, V> w[kGroupRows + 2];
#pragma unroll
    for (int t = 0; t < kGroupRows + 2; ++t) w[t] = ldv<R, V>(Pc + (size_t)(c0 + t) * ld);
#pragma unroll
    for (int r = 0; r < kGroupRows; ++r) {
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        const ab_pair<R> ce = ldc(ab + kb[r] + j + e);
#pragma unroll
        for (int v = 0; v < V; ++v) {
          apr[r][v] += ce.a * w[r + e].c[v].re;
          api[r][v] += ce.a * w[r + e].c[v].im;
          bpr[r][v] += ce.b * w[r + e].c[v].re;
          bpi[r][v] += ce.b * w[r + e].c[v].im;
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < kGroupRows; ++r)
#pragma unroll
    for (int v = 0; v < V; ++v)
      q[r].c[v] = {apr[r][v] - (sig[v].re * bpr[r][v] - sig[v].im * bpi[r][v]),
                   api[r][v] - (sig[v].re * bpi[r][v] + sig[v].im * bpr[r][v])};
}

constexpr int kNodeRows = 3;  // rows of a node triple (flags built on the host)
constexpr int kNodeChunk = 8;
constexpr int kSgsNodeChunk = 8;  // the same in the colour sweeps

// Complex-shifted sparse product of a node triple: rows i0 .. i0 + 2 with the
// same column list (checked on the host), so each input row is gathered once
// for the three rows: a third of the gathers of three generic rows.  Entries
// are taken in chunks of NC (the CSR padding covers the overrun of the
// last chunk; entries past the row end get zero coefficients and re-read row
// i0, whose values PZ replaces by zeros as in shifted_row); each row's entries
// are summed in entry order, as in shifted_row.
template <typename R, int V, bool PZ = false, int NC = kNodeChunk>
__device__ __forceinline__ void shifted_node(int i0, cptr<int> rowptr, cptr<int> col, cptr<ab_pair<R>> ab,
                                             const cx<R>* __restrict__ Pc, int ld, const cx<R> (&sig)[V],
                                             cvec<R, V> (&q)[kNodeRows]) {
  static_assert(NC <= kCsrPad, "chunk longer than the CSR padding");
  int kb[kNodeRows];
#pragma unroll
  for (int r = 0; r < kNodeRows; ++r) kb[r] = rowptr[i0 + r];
  const int m = rowptr[i0 + 1] - kb[0];
  R apr[kNodeRows][V] = {}, api[kNodeRows][V] = {}, bpr[kNodeRows][V] = {}, bpi[kNodeRows][V] = {};
#pragma unroll 1
  for (int j = 0; j < m; j += NC) {
    int jj[NC];
#pragma unroll
    for (int u = 0; u < NC; ++u) jj[u] = j + u < m ? col[kb[0] + j + u] : i0;
    cvec<R, V> x[NC];
#pragma unroll
    for (int u = 0; u < NC; ++u) x[u] = ldv<R, V>(Pc + (size_t)jj[u] * ld);
    if constexpr (PZ) {
#pragma unroll
      for (int u = 0; u < NC; ++u)
        if (j + u >= m) x[u] = cvec<R, V>{};
    }
#pragma unroll
    for (int r = 0; r < kNodeRows; ++r) {
#pragma unroll
      for (int u = 0; u < NC; ++u) {
        ab_pair<R> ce = ldc(ab + kb[r] + j + u);
        if (j + u >= m) ce = ab_pair<R>{0, 0};
#pragma unroll
        for (int v = 0; v < V; ++v) {
          apr[r][v] += ce.a * x[u].c[v].re;
          api[r][v] += ce.a * x[u].c[v].im;
          bpr[r][v] += ce.b * x[u].c[v].re;
          bpi[r][v] += ce.b * x[u].c[v].im;
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < kNodeRows; ++r)
#pragma unroll
    for (int v = 0; v < V; ++v)
      q[r].c[v] = {apr[r][v] - (sig[v].re * bpr[r][v] - sig[v].im * bpi[r][v]),
                   api[r][v] - (sig[v].re * bpi[r][v] + sig[v].im * bpr[r][v])};
}

// Block layout: a pencil's n x Kp block is stored tile by tile.  Tile t holds
// columns [t W, (t + 1) W) (W = 64 V, Kp a multiple of W) as an n x W row-major
// panel, so the rows a tile's kernels gather are W * 8 or W * 16 bytes apart
// whatever the number of columns.
__device__ __forceinline__ size_t tile_base(const Inst& I, int t, int V) {
  return I.blk + (size_t)t * (size_t)I.n * (WAVE * V);
}

// Loop header shared by the batched kernels: tile tg of pencil I.  cl0 is the
// lane's first column within the pencil (a multiple of V), cc0 that column
// clamped into the padded range, cg0 its global column; column v of the lane is
// real if cl0 + v < I.K.  FOR_TILES walks every tile; FOR_ACTIVE_TILES walks the
// list of tiles that had an active column at the last poll (iteration kernels).
#define FOR_TILE_LIST(b, p, V, COUNT, TG)                                    \
  for (int ti_ = 0; ti_ < (COUNT); ++ti_) {                                  \
    const int tg = (TG);                                                     \
    const Inst I = ldc(as_const((b).inst) + as_const((b).tile_inst)[tg]);    \
    const int cl0 = (tg - I.tile0) * (WAVE * (V)) + (p).lane * (V);          \
    const bool valid = cl0 < I.K;                                            \
    const int cc0 = min(cl0, I.Kp - (V));                                    \
    const int cg0 = I.col0 + cc0;                                            \
    const size_t tb = tile_base(I, tg - I.tile0, (V)) + (size_t)(p).lane * (V); \
    const size_t po = (size_t)blockIdx.x * (b).Ktot + I.col0 + (size_t)(tg - I.tile0) * (WAVE * (V));

#define FOR_TILES(b, p, V) FOR_TILE_LIST(b, p, V, (b).n_tiles, ti_)
#define FOR_ACTIVE_TILES(b, p, V) \
  FOR_TILE_LIST(b, p, V, as_const((const int*)(b).n_active)[0], as_const((const int*)(b).active)[ti_])

#define FOR_ROWS(b, p, I)                                               \
  for (int t_ = 0; t_ < (I).steps; ++t_) {                              \
    const int rb_ = step_block((I), (p), t_);                           \
    if (rb_ < 0) break;                                                 \
    const int r1_ = min((rb_ + 1) * (b).rows_per_block, (I).n);         \
    for (int pos = rb_ * (b).rows_per_block + (p).w; pos < r1_; pos += 4) {

#define END_ROWS \
  }              \
  }

// Row loop of the vector updates: a wavefront takes U of its rows at a time
// (positions q, q + 4, ..., in the order FOR_ROWS visits them), so that all
// their loads are issued before the first store.  ic[u] is row u's index clamped
// into the block (in bounds for loads); ok[u] says whether row u exists.
#define FOR_ROW_BATCH(b, p, I, U)                                             \
  for (int t_ = 0; t_ < (I).steps; ++t_) {                                    \
    const int rb_ = step_block((I), (p), t_);                                 \
    if (rb_ < 0) break;                                                       \
    const int r1_ = min((rb_ + 1) * (b).rows_per_block, (I).n);               \
    for (int q_ = rb_ * (b).rows_per_block + (p).w; q_ < r1_; q_ += 4 * (U)) { \
      int ic[U];                                                              \
      bool ok[U];                                                             \
      _Pragma("unroll") for (int u = 0; u < (U); ++u) {                       \
        ok[u] = q_ + 4 * u < r1_;                                             \
        ic[u] = ok[u] ? q_ + 4 * u : r1_ - 1;                                 \
      }

// Row loop of the sparse products for one tile: the workgroup's row blocks of
// pencil I; emit(i, q) receives row i's product.  When the row block is a
// multiple of 16 rows and the pencil has stencil groups, wavefront w takes the
// four consecutive positions rb * rows_per_block + 4 w + 16 k; if they hold one
// stencil group the shared-gather path serves them, else each is a generic row.
// Likewise with node triples and a multiple of 12 rows: wavefront w takes the
// three positions rb * rows_per_block + 3 w + 12 k.  Otherwise wavefront w takes
// every 4th position as in FOR_ROWS.
// MODE selects the shared-gather path compiled in (each adds registers to the
// kernel): kRowsGeneric none, kRowsQuads stencil groups, kRowsTriples node
// triples.  A pencil without that kind of row sets takes the generic rows.
constexpr int kRowsGeneric = 0, kRowsQuads = 1, kRowsTriples = 2;

template <typename R, int V, int MODE, typename Emit>
__device__ __forceinline__ void spmm_rows(const Batch& b, const WgPos& p, const Inst& I, const void* abv,
                                          const cx<R>* __restrict__ Pc, const cx<R> (&sig)[V], Emit&& emit) {
  const cptr<int> rowptr = as_const(I.rowptr), col = as_const(I.col);
  const cptr<ab_pair<R>> ab = as_const(static_cast<const ab_pair<R>*>(abv));
  const bool quads = MODE == kRowsQuads && I.groups && b.rows_per_block % (4 * kGroupRows) == 0;
  const bool triples = MODE == kRowsTriples && I.nodes && b.rows_per_block % (4 * kNodeRows) == 0;
  for (int t = 0; t < I.steps; ++t) {
    const int rb = step_block(I, p, t);
    if (rb < 0) break;
    const int r0 = rb * b.rows_per_block, r1 = min(r0 + b.rows_per_block, I.n);
    if (MODE == kRowsTriples && triples) {
      for (int q0 = r0 + kNodeRows * p.w; q0 < r1; q0 += 4 * kNodeRows) {
        const int cnt = min(kNodeRows, r1 - q0);
        const int i0 = I.sched ? as_const(I.sched)[q0] : q0;
        bool node = cnt == kNodeRows && i0 % kNodeRows == 0 && as_const(I.nodes)[i0 / kNodeRows] != 0;
        if (node && I.sched) {
#pragma unroll
          for (int u = 1; u < kNodeRows; ++u) node = node && as_const(I.sched)[q0 + u] == i0 + u;
        }
        if (node) {
          cvec<R, V> q[kNodeRows];
          shifted_node<R, V>(i0, rowptr, col, ab, Pc, WAVE * V, sig, q);
#pragma unroll
          for (int u = 0; u < kNodeRows; ++u) emit(i0 + u, q[u]);
          continue;
        }
        for (int u = 0; u < cnt; ++u) {
          const int i = I.sched ? as_const(I.sched)[q0 + u] : q0 + u;
          emit(i, shifted_row<R, V, kChunkShared<R>>(i, rowptr, col, ab, Pc, WAVE * V, sig));
        }
      }
    } else if (MODE == kRowsQuads && quads) {
      for (int q0 = r0 + kGroupRows * p.w; q0 < r1; q0 += 4 * kGroupRows) {
        const int cnt = min(kGroupRows, r1 - q0);
        const int i0 = I.sched ? as_const(I.sched)[q0] : q0;
        bool grp = cnt == kGroupRows && i0 % kGroupRows == 0 && as_const(I.groups)[i0 / kGroupRows] != 0;
        if (grp && I.sched) {
#pragma unroll
          for (int u = 1; u < kGroupRows; ++u) grp = grp && as_const(I.sched)[q0 + u] == i0 + u;
        }
        if (grp) {
          cvec<R, V> q[kGroupRows];
          shifted_group<R, V>(i0, rowptr, col, ab, Pc, WAVE * V, sig, q);
#pragma unroll
          for (int u = 0; u < kGroupRows; ++u) emit(i0 + u, q[u]);
          continue;
        }
        {
          for (int u = 0; u < cnt; ++u) {
            const int i = I.sched ? as_const(I.sched)[q0 + u] : q0 + u;
            emit(i, shifted_row<R, V, kChunkShared<R>>(i, rowptr, col, ab, Pc, WAVE * V, sig));
          }
        }
      }
    } else {
      for (int pos = r0 + p.w; pos < r1; pos += 4) {
        const int i = I.sched ? as_const(I.sched)[pos] : pos;
        emit(i, shifted_row<R, V, kChunk>(i, rowptr, col, ab, Pc, WAVE * V, sig));
      }
    }
  }
}

// The rows of spmm_rows in the same order, each with a zero product (the
// defect of a zero start sums its norms in the order of the product's rows).
template <typename R, int V, int MODE, typename Emit>
__device__ __forceinline__ void zero_rows(const Batch& b, const WgPos& p, const Inst& I, Emit&& emit) {
  const bool quads = MODE == kRowsQuads && I.groups && b.rows_per_block % (4 * kGroupRows) == 0;
  const bool triples = MODE == kRowsTriples && I.nodes && b.rows_per_block % (4 * kNodeRows) == 0;
  const int per = quads ? kGroupRows : triples ? kNodeRows : 1;
  const cvec<R, V> zero{};
  for (int t = 0; t < I.steps; ++t) {
    const int rb = step_block(I, p, t);
    if (rb < 0) break;
    const int r0 = rb * b.rows_per_block, r1 = min(r0 + b.rows_per_block, I.n);
    for (int q0 = r0 + per * p.w; q0 < r1; q0 += 4 * per) {
      const int cnt = min(per, r1 - q0);
      for (int u = 0; u < cnt; ++u) emit(I.sched ? as_const(I.sched)[q0 + u] : q0 + u, zero);
    }
  }
}

// The sparse-product kernels declare 4 wavefronts per SIMD (<= 128 VGPRs): the
// grid puts at most 4 workgroups of 4 wavefronts on a CU.
// v = S p_hat, partial (rhat, v)
template <typename R, int MODE>
__global__ __launch_bounds__(WG, 4) void k_spmm_v(Batch b, KrylovState<R> st, int* counter) {
  constexpr int V = LaneWidth<R>::V;
  const WgPos p = wg_pos(b.G);
  FOR_ACTIVE_TILES(b, p, V)
    cx<R> d[V] = {};
    if (tile_has<V>(st.flags, cg0, cl0, I.K, COL_ACTIVE, COL_ACTIVE)) {
      count_tile(counter);
      cx<R> sig[V];
#pragma unroll
      for (int v = 0; v < V; ++v) sig[v] = st.sigma_col[cg0 + v];
      spmm_rows<R, V, MODE>(b, p, I, I.ab, st.ph + tb, sig, [&](int i, const cvec<R, V>& q) {
        if (!valid) return;
        const size_t e = tb + (size_t)i * (WAVE * V);
        stv_nt<R, V>(st.v + e, q);
        if (st.rhat_cx) {  // conj(rhat) * v
          const cvec<R, V> rh = ldv_nt<R, V>(st.rhat_cx + e);
#pragma unroll
          for (int v = 0; v < V; ++v) {
            d[v].re += rh.c[v].re * q.c[v].re + rh.c[v].im * q.c[v].im;
            d[v].im += rh.c[v].re * q.c[v].im - rh.c[v].im * q.c[v].re;
          }
        } else {
#pragma unroll
          for (int v = 0; v < V; ++v) {
            const R rh = st.rhat[I.rl + (size_t)i * I.L + col_rhs(cc0 + v, I.L, I.N, I.rmaj)];
            d[v].re += rh * q.c[v].re;
            d[v].im += rh * q.c[v].im;
          }
        }
      });
    }
    wg_store_partial_cx<R, V>(d, p.w, p.lane, cl0, I.K, st.part_a + po);
  }
}

// t = S s_hat, partials (t, s) = t^H s and (t, t)
template <typename R, int MODE>
__global__ __launch_bounds__(WG, 4) void k_spmm_t(Batch b, KrylovState<R> st, int* counter) {
  constexpr int V = LaneWidth<R>::V;
  const WgPos p = wg_pos(b.G);
  FOR_ACTIVE_TILES(b, p, V)
    cx<R> ts[V] = {};
    R tt[V] = {};
    if (tile_has<V>(st.flags, cg0, cl0, I.K, COL_ACTIVE, COL_ACTIVE)) {
      count_tile(counter);
      cx<R> sig[V];
#pragma unroll
      for (int v = 0; v < V; ++v) sig[v] = st.sigma_col[cg0 + v];
      spmm_rows<R, V, MODE>(b, p, I, I.ab, st.sh + tb, sig, [&](int i, const cvec<R, V>& tv) {
        if (valid) {
          const size_t e = tb + (size_t)i * (WAVE * V);
          stv_nt<R, V>(st.t + e, tv);
          cvec<R, V> sv;
          if (st.s) {
            sv = ldv_nt<R, V>(st.s + e);
          } else {
            const cvec<R, V> shv = ldv<R, V>(st.sh + e);
#pragma unroll
            for (int v = 0; v < V; ++v)
              sv.c[v] = cmul(st.d[I.dn + (size_t)i * I.N + col_pole(cc0 + v, I.L, I.N, I.rmaj)], shv.c[v]);
          }
#pragma unroll
          for (int v = 0; v < V; ++v) {
            const cx<R> t = tv.c[v], s = sv.c[v];
            ts[v].re += t.re * s.re + t.im * s.im;  // conj(t) * s
            ts[v].im += t.re * s.im - t.im * s.re;
            tt[v] += t.re * t.re + t.im * t.im;
          }
        }
      });
    }
    wg_store_partial_cx<R, V>(ts, p.w, p.lane, cl0, I.K, st.part_a + po);
    wg_store_partial<R, V>(tt, p.w, p.lane, cl0, I.K, st.part_b + po);
  }
}

// p = r + beta (p - omega v)  (first iteration: p = r).
// Jacobi batch: p itself is not stored; p_hat = p / d with p = d p_hat.
// Batch with ILU(0) or block-Jacobi pencils: p is stored; their kernels form
// p_hat for those pencils, and Jacobi pencils of the same batch form
// p_hat = p / d here.  Columns that are not active keep their values.
template <typename R>
__global__ __launch_bounds__(WG, 4) void k_update_p(Batch b, KrylovState<R> st, int first, int* counter) {
  constexpr int V = LaneWidth<R>::V;
  const WgPos p = wg_pos(b.G);
  FOR_ACTIVE_TILES(b, p, V)
    (void)po;
    if (!tile_has<V>(st.flags, cg0, cl0, I.K, COL_ACTIVE, COL_ACTIVE)) continue;
    count_tile(counter);
    int f[V];
    lane_flags<V>(st.flags, cg0, cl0, I.K, f);
    bool any = false;
    int pole[V];
    cx<R> beta[V], omega[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      any |= f[v] == COL_ACTIVE;
      pole[v] = col_pole(cc0 + v, I.L, I.N, I.rmaj);
      beta[v] = st.beta[cg0 + v];
      omega[v] = st.omega[cg0 + v];
    }
    if (!any) continue;
    bool keep = false;  // some column of the lane is not updated: its old values are stored back
#pragma unroll
    for (int v = 0; v < V; ++v) keep |= f[v] != COL_ACTIVE;
    const bool jac_here = !I.ilu && !I.bjac;
    constexpr int kRowBatch = 4;
    FOR_ROW_BATCH(b, p, I, kRowBatch)
      size_t e[kRowBatch];
      cvec<R, V> r[kRowBatch], pv[kRowBatch], vv[kRowBatch], ph[kRowBatch];
#pragma unroll
      for (int u = 0; u < kRowBatch; ++u) {
        e[u] = tb + (size_t)ic[u] * (WAVE * V);
        r[u] = ldv<R, V>(st.r + e[u]);
        if (!first || keep) pv[u] = ldv<R, V>(st.p ? st.p + e[u] : st.ph + e[u]);
        if (!first) vv[u] = ldv<R, V>(st.v + e[u]);
        if (st.p && jac_here && keep) ph[u] = ldv<R, V>(st.ph + e[u]);
      }
#pragma unroll
      for (int u = 0; u < kRowBatch; ++u) {
        if (!ok[u]) continue;
        const size_t de = I.dn + (size_t)ic[u] * I.N;
        if (st.p) {
#pragma unroll
          for (int v = 0; v < V; ++v) {
            if (f[v] != COL_ACTIVE) continue;
            cx<R> pn = r[u].c[v];
            if (!first) pn = cadd(pn, cmul(beta[v], csub(pv[u].c[v], cmul(omega[v], vv[u].c[v]))));
            pv[u].c[v] = pn;
            if (jac_here) ph[u].c[v] = cmul(pn, st.dinv[de + pole[v]]);
          }
          stv<R, V>(st.p + e[u], pv[u]);
          if (jac_here) stv<R, V>(st.ph + e[u], ph[u]);
        } else {  // pv holds p_hat
#pragma unroll
          for (int v = 0; v < V; ++v) {
            if (f[v] != COL_ACTIVE) continue;
            cx<R> pn = r[u].c[v];
            if (!first)
              pn = cadd(pn, cmul(beta[v], csub(cmul(st.d[de + pole[v]], pv[u].c[v]), cmul(omega[v], vv[u].c[v]))));
            pv[u].c[v] = cmul(pn, st.dinv[de + pole[v]]);
          }
          stv<R, V>(st.ph + e[u], pv[u]);
        }
      }
    END_ROWS
  }
}

// s = r - alpha v (Jacobi batch: s_hat = s / d is stored instead; in a batch
// with ILU(0) or block-Jacobi pencils s is stored, plus s_hat = s / d for its
// Jacobi pencils) ; partial |s|^2
template <typename R>
__global__ __launch_bounds__(WG, 4) void k_update_s(Batch b, KrylovState<R> st, int* counter) {
  constexpr int V = LaneWidth<R>::V;
  const WgPos p = wg_pos(b.G);
  FOR_ACTIVE_TILES(b, p, V)
    R ss[V] = {};
    if (tile_has<V>(st.flags, cg0, cl0, I.K, COL_ACTIVE, COL_ACTIVE)) {
      count_tile(counter);
      int f[V];
      lane_flags<V>(st.flags, cg0, cl0, I.K, f);
      bool any = false;
      int pole[V];
      cx<R> alpha[V];
#pragma unroll
      for (int v = 0; v < V; ++v) {
        any |= f[v] == COL_ACTIVE;
        pole[v] = col_pole(cc0 + v, I.L, I.N, I.rmaj);
        alpha[v] = st.alpha[cg0 + v];
      }
      if (any) {
        bool keep = false;
#pragma unroll
        for (int v = 0; v < V; ++v) keep |= f[v] != COL_ACTIVE;
        const bool jac_here = !st.s || (!I.ilu && !I.bjac);
        constexpr int kRowBatch = 4;
        FOR_ROW_BATCH(b, p, I, kRowBatch)
          size_t e[kRowBatch];
          cvec<R, V> r[kRowBatch], vv[kRowBatch], sv[kRowBatch], sh[kRowBatch];
#pragma unroll
          for (int u = 0; u < kRowBatch; ++u) {
            e[u] = tb + (size_t)ic[u] * (WAVE * V);
            r[u] = ldv<R, V>(st.r + e[u]);
            vv[u] = ldv<R, V>(st.v + e[u]);
            if (st.s && keep) sv[u] = ldv<R, V>(st.s + e[u]);
            if (jac_here && keep) sh[u] = ldv<R, V>(st.sh + e[u]);
          }
#pragma unroll
          for (int u = 0; u < kRowBatch; ++u) {
            if (!ok[u]) continue;
            const size_t de = I.dn + (size_t)ic[u] * I.N;
#pragma unroll
            for (int v = 0; v < V; ++v) {
              if (f[v] != COL_ACTIVE) continue;
              const cx<R> s = csub(r[u].c[v], cmul(alpha[v], vv[u].c[v]));
              ss[v] += s.re * s.re + s.im * s.im;
              sv[u].c[v] = s;
              if (jac_here) sh[u].c[v] = cmul(s, st.dinv[de + pole[v]]);
            }
            if (st.s) stv<R, V>(st.s + e[u], sv[u]);
            if (jac_here) stv<R, V>(st.sh + e[u], sh[u]);
          }
        END_ROWS
      }
    }
    wg_store_partial<R, V>(ss, p.w, p.lane, cl0, I.K, st.part_b + po);
  }
}

// x += alpha p_hat + omega s_hat ; r = s - omega t ; partials (rhat, r), |r|^2
// Columns that converged at the half step take x += alpha p_hat only.
template <typename R>
__global__ __launch_bounds__(WG, 4) void k_update_x(Batch b, KrylovState<R> st, int first, int* counter) {
  constexpr int V = LaneWidth<R>::V;
  const WgPos p = wg_pos(b.G);
  FOR_ACTIVE_TILES(b, p, V)
    cx<R> rd[V] = {};
    R nn[V] = {};
    if (tile_has<V>(st.flags, cg0, cl0, I.K, COL_ACTIVE, COL_HALF_PENDING)) {
      count_tile(counter);
      int f[V];
      lane_flags<V>(st.flags, cg0, cl0, I.K, f);
      bool act[V], half[V], any = false;
      int pole[V];
      cx<R> alpha[V], omega[V];
#pragma unroll
      for (int v = 0; v < V; ++v) {
        act[v] = f[v] == COL_ACTIVE;
        half[v] = f[v] == COL_HALF_PENDING;
        any |= act[v] || half[v];
        pole[v] = col_pole(cc0 + v, I.L, I.N, I.rmaj);
        alpha[v] = st.alpha[cg0 + v];
        omega[v] = act[v] ? st.omega[cg0 + v] : cx<R>{0, 0};
      }
      if (any) {
        bool keep_x = false, keep_r = false, any_act = false;
#pragma unroll
        for (int v = 0; v < V; ++v) {
          keep_x |= !act[v] && !half[v];
          keep_r |= !act[v];
          any_act |= act[v];
        }
        constexpr int kRowBatch = 2;
        FOR_ROW_BATCH(b, p, I, kRowBatch)
          size_t e[kRowBatch];
          cvec<R, V> x[kRowBatch], ph[kRowBatch], sh[kRowBatch], t[kRowBatch], r[kRowBatch], sv[kRowBatch],
              rh[kRowBatch];
          cx<R> dg[kRowBatch][V];
          R rr[kRowBatch][V];
#pragma unroll
          for (int u = 0; u < kRowBatch; ++u) {
            e[u] = tb + (size_t)ic[u] * (WAVE * V);
            if (!first || keep_x) x[u] = ldv<R, V>(st.x + e[u]);
            ph[u] = ldv<R, V>(st.ph + e[u]);
            if (any_act) {
              sh[u] = ldv<R, V>(st.sh + e[u]);
              t[u] = ldv<R, V>(st.t + e[u]);
              if (st.s) {
                sv[u] = ldv<R, V>(st.s + e[u]);
              } else {
                const size_t de = I.dn + (size_t)ic[u] * I.N;
#pragma unroll
                for (int v = 0; v < V; ++v) dg[u][v] = st.d[de + pole[v]];
              }
              if (st.rhat_cx) {
                rh[u] = ldv<R, V>(st.rhat_cx + e[u]);
              } else {
#pragma unroll
                for (int v = 0; v < V; ++v) rr[u][v] = st.rhat[I.rl + (size_t)ic[u] * I.L + col_rhs(cc0 + v, I.L, I.N, I.rmaj)];
              }
            }
            if (keep_r) r[u] = ldv<R, V>(st.r + e[u]);
          }
#pragma unroll
          for (int u = 0; u < kRowBatch; ++u) {
            if (!ok[u]) continue;
#pragma unroll
            for (int v = 0; v < V; ++v) {
              if (first && (act[v] || half[v] || !keep_x)) x[u].c[v] = {0, 0};
              if (!act[v] && !half[v]) continue;
              x[u].c[v] = cadd(x[u].c[v], cmul(alpha[v], ph[u].c[v]));
              if (!act[v]) continue;
              x[u].c[v] = cadd(x[u].c[v], cmul(omega[v], sh[u].c[v]));
              const cx<R> s = st.s ? sv[u].c[v] : cmul(dg[u][v], sh[u].c[v]);
              const cx<R> rv = csub(s, cmul(omega[v], t[u].c[v]));
              r[u].c[v] = rv;
              if (st.rhat_cx) {
                rd[v].re += rh[u].c[v].re * rv.re + rh[u].c[v].im * rv.im;
                rd[v].im += rh[u].c[v].re * rv.im - rh[u].c[v].im * rv.re;
              } else {
                rd[v].re += rr[u][v] * rv.re;
                rd[v].im += rr[u][v] * rv.im;
              }
              nn[v] += rv.re * rv.re + rv.im * rv.im;
            }
            if (any_act) stv<R, V>(st.r + e[u], r[u]);
            stv<R, V>(st.x + e[u], x[u]);
          }
        END_ROWS
      }
    }
    wg_store_partial_cx<R, V>(rd, p.w, p.lane, cl0, I.K, st.part_a + po);
    wg_store_partial<R, V>(nn, p.w, p.lane, cl0, I.K, st.part_b + po);
  }
}

// x = 0, r = f (broadcast over poles); partials of ||f||^2
template <typename R>
__global__ __launch_bounds__(WG) void k_init(Batch b, KrylovState<R> st, const R* __restrict__ F) {
  constexpr int V = LaneWidth<R>::V;
  const WgPos p = wg_pos(b.G);
  FOR_TILES(b, p, V)
    R nn[V] = {};
    if (valid) {
      FOR_ROWS(b, p, I)
        const int i = pos;
        const size_t e = tb + (size_t)i * (WAVE * V);
        cvec<R, V> r, x;
#pragma unroll
        for (int v = 0; v < V; ++v) {
          const R fv = cl0 + v < I.K ? F[I.rl + (size_t)i * I.L + col_rhs(cc0 + v, I.L, I.N, I.rmaj)] : R(0);
          r.c[v] = {fv, 0};
          x.c[v] = {0, 0};
          nn[v] += fv * fv;
        }
        stv<R, V>(st.r + e, r);
        stv<R, V>(st.x + e, x);
      END_ROWS
    }
    wg_store_partial<R, V>(nn, p.w, p.lane, cl0, I.K, st.part_b + po);
  }
}

// ---------------------------------------------------------------------------
// Per-column scalar kernels: one 256-thread block per global tile, each lane
// handling V columns.  The sum over the G partials is split across the 4
// wavefronts (slots k = w, w + 4, ..., loads kept in flight by unrolling) and
// combined in a fixed order; wavefront 0 then applies the update.  Slot k is row
// block slot k >> 3 of XCD k & 7; its partial sits in the row of the workgroup
// that the pencil's rotation gave that slot.  Summing in slot order makes the
// result independent of the grid size and of the rotation: a pencil's sums are
// the same alone and in a batch (a larger grid only appends zero partials).
__device__ __forceinline__ size_t slot_partial(int k, int per, int rot) {
  int q = (k >> 3) - rot;
  if (q < 0) q += per;
  return (size_t)(8 * q + (k & 7));
}

// Which slots of a pencil's partial sums to add.  A workgroup that owns none
// of the pencil's rows stores zeros, and a sum that starts at +0 is not changed
// by adding +0, so skipping those slots leaves every sum bit for bit as it was.
//   kind 0: every slot k < G of the grid (row slot_partial(k, G / 8, rot));
//   kind 1: the same slots, those whose first row block (step_block) exists;
//   kind 2: the colour shares of the SGS sweeps: share g < count sits in the
//           row of workgroup (x = g / per, q = g % per) of the sweep grid (per
//           workgroups per XCD).  Shares are summed in share order, which does
//           not depend on the sweep grid, so a pencil's sums are the same alone
//           and in a batch.
struct SlotSet {
  int kind = 0;
  int slab = 0, nrb = 0;  // kind 1
  int count = 0, per = 1;  // kind 2
  __device__ bool live(int k) const {
    if (kind != 1) return true;
    const int j = k >> 3;
    return j < slab && (k & 7) * slab + j < nrb;
  }
};

__device__ __forceinline__ SlotSet rows_live(const Inst& I) {
  SlotSet l;
  l.kind = 1;
  l.slab = I.slab;
  l.nrb = I.nrb;
  return l;
}

__device__ __forceinline__ SlotSet sweep_shares(const Inst& I, const Batch& b) {
  SlotSet l;
  l.kind = 2;
  l.count = I.sgs_wgs;
  l.per = b.Gs >> 3;
  return l;
}

// Column sums of the partials: wavefront w of the block's nw (up to 16) adds
// slots w, w + nw, ... in slot order (the live ones), then the nw sums are
// added in wavefront order (the order depends only on the block size).
constexpr int kMaxScWaves = 16;
// threads of the COCG scalar kernels (one block per column tile: the G partials
// of each column are read by 16 wavefronts)
constexpr int kScWG = kMaxScWaves * WAVE;
__device__ __forceinline__ size_t slot_row(const SlotSet& s, int k, int per, int rot) {
  return s.kind == 2 ? (size_t)(8 * (k % s.per) + k / s.per) : slot_partial(k, per, rot);
}

template <typename T>
__device__ __forceinline__ T block_col_sum(const T* __restrict__ part, int G, int rot, int Ktot, int c,
                                           bool valid, const SlotSet& set = SlotSet{}) {
  __shared__ T red[kMaxScWaves][WAVE];
  const int w = wave_id(), lane = lane_id(), per = G >> 3, nw = blockDim.x / WAVE;
  const int cnt = set.kind == 2 ? set.count : G;
  T acc = 0;
  if (valid) {
    // a skipped slot adds +0 (its load is redirected to row 0, a cached line):
    // the loads stay unconditional, so the unrolled ones are all in flight
#pragma unroll 8
    for (int k = w; k < cnt; k += nw) {
      const bool on = set.live(k);
      const T v = part[(on ? slot_row(set, k, per, rot) : 0) * Ktot + c];
      acc += on ? v : T(0);
    }
  }
  red[w][lane] = acc;
  __syncthreads();
  T tot = red[0][lane];
  for (int i = 1; i < nw; ++i) tot += red[i][lane];
  __syncthreads();
  return tot;
}

template <typename R>
__device__ __forceinline__ cx<R> block_col_sum_cx(const cx<R>* part, int G, int rot, int Ktot, int c,
                                                  bool valid, const SlotSet& set = SlotSet{}) {
  __shared__ R rr[kMaxScWaves][WAVE], ri[kMaxScWaves][WAVE];
  const int w = wave_id(), lane = lane_id(), per = G >> 3, nw = blockDim.x / WAVE;
  const int cnt = set.kind == 2 ? set.count : G;
  R ar = 0, ai = 0;
  if (valid) {
#pragma unroll 8
    for (int k = w; k < cnt; k += nw) {
      const bool on = set.live(k);
      const cx<R> v = part[(on ? slot_row(set, k, per, rot) : 0) * Ktot + c];
      ar += on ? v.re : R(0);
      ai += on ? v.im : R(0);
    }
  }
  rr[w][lane] = ar;
  ri[w][lane] = ai;
  __syncthreads();
  cx<R> tot = {rr[0][lane], ri[0][lane]};
  for (int i = 1; i < nw; ++i) {
    tot.re += rr[i][lane];
    tot.im += ri[i][lane];
  }
  __syncthreads();
  return tot;
}

template <typename R>
__device__ __forceinline__ bool cfinite(cx<R> z) { return isfinite(z.re) && isfinite(z.im); }

// lane's first column (cl0), its global column (cg0), and the wavefront that
// applies the per-column updates
#define SC_PROLOGUE(V)                                                        \
  const Inst I = ldc(as_const(b.inst) + as_const(b.tile_inst)[blockIdx.x]);   \
  const int cl0 = (blockIdx.x - I.tile0) * (WAVE * (V)) + lane_id() * (V);    \
  const int cg0 = I.col0 + min(cl0, I.Kp - (V));                              \
  const bool lead = wave_id() == 0;

// alpha = rho / (rhat, v)
template <typename R>
__global__ __launch_bounds__(WG) void k_sc_alpha(Batch b, KrylovState<R> st) {
  constexpr int V = LaneWidth<R>::V;
  SC_PROLOGUE(V)
  if (!tile_has<V>(st.flags, cg0, cl0, I.K, COL_ACTIVE, COL_ACTIVE)) return;
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const int c = cg0 + v;
    const bool ok = cl0 + v < I.K;
    const cx<R> rv = block_col_sum_cx(st.part_a, b.G, I.rot, b.Ktot, c, ok);
    if (!lead || !ok || st.flags[c] != COL_ACTIVE) continue;
    const cx<R> rho = st.rho[c];
    if ((rv.re == 0 && rv.im == 0) || (rho.re == 0 && rho.im == 0) || !cfinite(rv)) {
      st.flags[c] = COL_BREAKDOWN;
      continue;
    }
    st.alpha[c] = cdiv(rho, rv);
    st.iters[c] += 1;
  }
}

// half-step test ||s|| <= tol ||f||
template <typename R>
__global__ __launch_bounds__(WG) void k_sc_half(Batch b, KrylovState<R> st, R tol) {
  constexpr int V = LaneWidth<R>::V;
  SC_PROLOGUE(V)
  if (!tile_has<V>(st.flags, cg0, cl0, I.K, COL_ACTIVE, COL_ACTIVE)) return;
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const int c = cg0 + v;
    const bool ok = cl0 + v < I.K;
    const R sn = sqrt(block_col_sum(st.part_b, b.G, I.rot, b.Ktot, c, ok));
    if (!lead || !ok || st.flags[c] != COL_ACTIVE) continue;
    if (sn <= (st.tolc ? st.tolc[c] : tol) * st.fnorm[c]) {
      st.flags[c] = COL_HALF_PENDING;
      st.rnorm[c] = sn;
    }
  }
}

// omega = (t, s) / (t, t)
template <typename R>
__global__ __launch_bounds__(WG) void k_sc_omega(Batch b, KrylovState<R> st) {
  constexpr int V = LaneWidth<R>::V;
  SC_PROLOGUE(V)
  if (!tile_has<V>(st.flags, cg0, cl0, I.K, COL_ACTIVE, COL_ACTIVE)) return;
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const int c = cg0 + v;
    const bool ok = cl0 + v < I.K;
    const cx<R> ts = block_col_sum_cx(st.part_a, b.G, I.rot, b.Ktot, c, ok);
    const R tt = block_col_sum(st.part_b, b.G, I.rot, b.Ktot, c, ok);
    if (!lead || !ok || st.flags[c] != COL_ACTIVE) continue;
    if (tt == 0 || !isfinite(tt)) {
      st.flags[c] = COL_BREAKDOWN;
      continue;
    }
    st.omega[c] = {ts.re / tt, ts.im / tt};
  }
}

// rho_new = (rhat, r); ||r|| test; beta = (rho_new / rho)(alpha / omega)
template <typename R>
__global__ __launch_bounds__(WG) void k_sc_beta(Batch b, KrylovState<R> st, R tol, int maxit) {
  constexpr int V = LaneWidth<R>::V;
  SC_PROLOGUE(V)
  if (!tile_has<V>(st.flags, cg0, cl0, I.K, COL_ACTIVE, COL_HALF_PENDING)) return;
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const int c = cg0 + v;
    const bool ok = cl0 + v < I.K;
    const cx<R> rn = block_col_sum_cx(st.part_a, b.G, I.rot, b.Ktot, c, ok);
    const R nn = sqrt(block_col_sum(st.part_b, b.G, I.rot, b.Ktot, c, ok));
    if (!lead || !ok) continue;
    const int f = st.flags[c];
    if (f == COL_HALF_PENDING) {
      st.flags[c] = COL_HALF_CONVERGED;
      continue;
    }
    if (f != COL_ACTIVE) continue;
    st.rnorm[c] = nn;
    if (nn <= (st.tolc ? st.tolc[c] : tol) * st.fnorm[c]) {
      st.flags[c] = COL_CONVERGED;
      continue;
    }
    if (st.iters[c] >= maxit) {
      st.flags[c] = COL_MAXIT;
      continue;
    }
    const cx<R> om = st.omega[c];
    if ((om.re == 0 && om.im == 0) || !cfinite(rn)) {
      st.flags[c] = COL_BREAKDOWN;
      continue;
    }
    st.beta[c] = cmul(cdiv(rn, st.rho[c]), cdiv(st.alpha[c], om));
    st.rho[c] = rn;
  }
}

// Per-column start values; padding columns (past K) are marked converged.
template <typename R>
__global__ __launch_bounds__(WG) void k_init_scalars(Batch b, KrylovState<R> st) {
  constexpr int V = LaneWidth<R>::V;
  SC_PROLOGUE(V)
  if (threadIdx.x == 0) {  // every tile starts on the active list
    b.active[blockIdx.x] = blockIdx.x;
    if (blockIdx.x == 0) b.n_active[0] = b.n_tiles;
  }
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const int c = cg0 + v;
    const bool ok = cl0 + v < I.K;
    const R nn = block_col_sum(st.part_b, b.G, I.rot, b.Ktot, c, ok);
    if (!lead || cl0 + v >= I.Kp) continue;
    st.fnorm[c] = sqrt(nn);
    st.rnorm[c] = sqrt(nn);
    st.rho[c] = {nn, 0};
    st.alpha[c] = {1, 0};
    st.omega[c] = {1, 0};
    st.beta[c] = {0, 0};
    st.iters[c] = 0;
    st.flags[c] = (nn == 0 || !ok) ? COL_CONVERGED : COL_ACTIVE;
  }
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
  if (c >= I.K) return;
  const cx<R>* f = static_cast<const cx<R>*>(I.ilu) + (size_t)col_pole(c, I.L, I.N, I.rmaj) * I.nnz;
  constexpr int W = WAVE * LaneWidth<R>::V;
  const size_t col_base = tile_base(I, c / W, LaneWidth<R>::V) + c % W;
  const cx<R>* src = in + col_base;
  cx<R>* dst = out + col_base;
  const size_t ld = W;
  cx<R> prev = {0, 0};
  for (int i = 0; i < I.n; ++i) {
    cx<R> y = src[(size_t)i * ld];
    const int kd = I.diagpos[i];
    for (int k = I.rowptr[i]; k < kd; ++k) {
      const int j = I.col[k];
      const cx<R> yj = (j == i - 1) ? prev : dst[(size_t)j * ld];
      y = csub(y, cmul(f[k], yj));
    }
    dst[(size_t)i * ld] = y;
    prev = y;
  }
  prev = {0, 0};
  for (int i = I.n - 1; i >= 0; --i) {
    cx<R> z = dst[(size_t)i * ld];
    const int kd = I.diagpos[i];
    for (int k = kd + 1; k < I.rowptr[i + 1]; ++k) {
      const int j = I.col[k];
      const cx<R> zj = (j == i + 1) ? prev : dst[(size_t)j * ld];
      z = csub(z, cmul(f[k], zj));
    }
    z = cmul(z, f[kd]);
    dst[(size_t)i * ld] = z;
    prev = z;
  }
}

// out = M^{-1} in for node block Jacobi: unknowns 3k, 3k+1, 3k+2 form node k and
// M_k^{-1} (3x3, per pole) multiplies them.  One thread per (node, V columns);
// only active columns of pencils that use block Jacobi are written.
template <typename R>
__global__ __launch_bounds__(WG) void k_bjac_apply(Batch b, const int* __restrict__ flags,
                                                  const cx<R>* __restrict__ in, cx<R>* __restrict__ out) {
  constexpr int V = LaneWidth<R>::V;
  const WgPos p = wg_pos(b.G);
  FOR_ACTIVE_TILES(b, p, V)
    (void)po;
    if (!I.bjac || !valid) continue;
    int f[V];
    lane_flags<V>(flags, cg0, cl0, I.K, f);
    bool any = false;
#pragma unroll
    for (int v = 0; v < V; ++v) any |= f[v] == COL_ACTIVE;
    if (!any) continue;
    bool keep = false;
#pragma unroll
    for (int v = 0; v < V; ++v) keep |= f[v] != COL_ACTIVE;
    const int nodes = I.n / 3;
    const size_t stride = WAVE * V;
    for (int k = blockIdx.x * 4 + p.w; k < nodes; k += b.G * 4) {
      const size_t e0 = tb + (size_t)(3 * k) * stride;
      const cvec<R, V> x0 = ldv<R, V>(in + e0), x1 = ldv<R, V>(in + e0 + stride), x2 = ldv<R, V>(in + e0 + 2 * stride);
      cvec<R, V> y[3];
      if (keep)
#pragma unroll
        for (int r = 0; r < 3; ++r) y[r] = ldv<R, V>(out + e0 + r * stride);
#pragma unroll
      for (int v = 0; v < V; ++v) {
        if (f[v] != COL_ACTIVE) continue;
        const cx<R>* m = static_cast<const cx<R>*>(I.bjac) +
                         ((size_t)col_pole(cc0 + v, I.L, I.N, I.rmaj) * nodes + (size_t)k) * 9;
#pragma unroll
        for (int r = 0; r < 3; ++r)
          y[r].c[v] = cadd(cadd(cmul(m[3 * r], x0.c[v]), cmul(m[3 * r + 1], x1.c[v])), cmul(m[3 * r + 2], x2.c[v]));
      }
#pragma unroll
      for (int r = 0; r < 3; ++r) stv<R, V>(out + e0 + r * stride, y[r]);
    }
  }
}

int* LaunchTimer::begin(hipStream_t s, int kind, double tile_bytes, double fixed, double share, int grid) {
  if (used >= capacity || used >= 512) return nullptr;
  recs[used] = {kind, tile_bytes, fixed, share, grid};
  (void)hipEventRecord(events[2 * used], s);
  return d_counts + used;
}
void LaunchTimer::end(hipStream_t s) {
  (void)hipEventRecord(events[2 * used + 1], s);
  ++used;
}

template <typename R>
void launch_iteration(hipStream_t s, const Batch& b, const KrylovState<R>& st, R tol, int maxit, bool first,
                      int precs, LaunchTimer* tm, const IterBytes& by) {
  const bool ilu = precs & 1, bjac = precs & 2;
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
  if (bjac) k_bjac_apply<R><<<grid, blk, 0, s>>>(b, st.flags, st.p, st.ph);
  // v = S p_hat: gather p_hat once, write v, read rhat; the merged CSR once per launch
  c = tm ? tm->begin(s, 0, 2 * by.blk + by.rhat, by.matrix) : nullptr;
  if (b.groups == kRowsQuads)
    k_spmm_v<R, kRowsQuads><<<grid, blk, 0, s>>>(b, st, c);
  else if (b.groups == kRowsTriples)
    k_spmm_v<R, kRowsTriples><<<grid, blk, 0, s>>>(b, st, c);
  else
    k_spmm_v<R, kRowsGeneric><<<grid, blk, 0, s>>>(b, st, c);
  if (c) tm->end(s);
  k_sc_alpha<R><<<cgrid, cblk, 0, s>>>(b, st);
  c = tm ? tm->begin(s, 1, 3 * by.blk + (jac ? by.diag : 0), 0) : nullptr;
  k_update_s<R><<<grid, blk, 0, s>>>(b, st, c);
  if (c) tm->end(s);
  k_sc_half<R><<<cgrid, cblk, 0, s>>>(b, st, tol);
  if (ilu) k_ilu_apply<R><<<igrid, iblk, 0, s>>>(b, st.flags, st.s, st.sh);
  if (bjac) k_bjac_apply<R><<<grid, blk, 0, s>>>(b, st.flags, st.s, st.sh);
  c = tm ? tm->begin(s, 0, (jac ? 2 : 3) * by.blk + (jac ? by.diag : 0), by.matrix) : nullptr;
  if (b.groups == kRowsQuads)
    k_spmm_t<R, kRowsQuads><<<grid, blk, 0, s>>>(b, st, c);
  else if (b.groups == kRowsTriples)
    k_spmm_t<R, kRowsTriples><<<grid, blk, 0, s>>>(b, st, c);
  else
    k_spmm_t<R, kRowsGeneric><<<grid, blk, 0, s>>>(b, st, c);
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
  const int tw = WAVE * b.V;
  int base = 0, ncols = 0;
  for (int t0 = 0; t0 < b.n_tiles; t0 += 256) {
    const int t = t0 + (int)threadIdx.x;
    int act = 0, cnt = 0;
    if (t < b.n_tiles) {
      const Inst I = b.inst[b.tile_inst[t]];
      const int c0 = I.col0 + (t - I.tile0) * tw;
      const int c1 = min(c0 + tw, I.col0 + I.K);
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
// Mixed precision: FP64 defect R = F - S Y and the FP32 <-> FP64 transfers.  The
// batch is the FP32 one, so a lane owns kMixedV adjacent columns.
constexpr int kMixedV = LaneWidth<float>::V;

// true if some column of the tile has scale > 0 (has not met its target)
template <int V>
__device__ __forceinline__ bool tile_open(const double* scale, int cg0, int cl0, int K) {
  bool open = false;
#pragma unroll
  for (int v = 0; v < V; ++v) open |= cl0 + v < K && scale[cg0 + v] > 0;
  return __any(open);
}

template <int MODE>
__global__ __launch_bounds__(WG) void k_defect(Batch b, const cx<double>* __restrict__ sigma_col,
                                              const double* __restrict__ F, const cx<double>* __restrict__ Y,
                                              cx<double>* __restrict__ Rout, double* __restrict__ part,
                                              const double* __restrict__ scale) {
  constexpr int V = kMixedV;
  const WgPos p = wg_pos(b.G);
  FOR_TILES(b, p, V)
    if (Y && !tile_open<V>(scale, cg0, cl0, I.K)) continue;  // every column already met its target
    cx<double> sig[V];
#pragma unroll
    for (int v = 0; v < V; ++v) sig[v] = sigma_col[cg0 + v];
    double nn[V] = {};
    auto emit = [&](int i, const cvec<double, V>& q) {
      cvec<double, V> r;
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const double f = cl0 + v < I.K ? F[I.rl + (size_t)i * I.L + col_rhs(cc0 + v, I.L, I.N, I.rmaj)] : 0.0;
        r.c[v] = Y ? cx<double>{f - q.c[v].re, -q.c[v].im} : cx<double>{f, 0.0};
        if (cl0 + v >= I.K) r.c[v] = {0.0, 0.0};
        // explicit fused steps: the zero-product copy of this code (zero_rows)
        // and the product copy then round |r|^2 alike (no contraction choice)
        nn[v] = fma(r.c[v].re, r.c[v].re, fma(r.c[v].im, r.c[v].im, nn[v]));
      }
      if (Y && valid) {
        const size_t e = tb + (size_t)i * (WAVE * V);
#pragma unroll
        for (int v = 0; v < V; ++v) Rout[e + v] = r.c[v];
      }
    };
    if (Y)
      spmm_rows<double, V, MODE>(b, p, I, I.ab64, Y + tb, sig, emit);
    else
      zero_rows<double, V, MODE>(b, p, I, emit);
    wg_store_partial<double, V>(nn, p.w, p.lane, cl0, I.K, part + po);
  }
}

void launch_defect(hipStream_t s, const Batch& b, const cx<double>* sigma_col, const double* F,
                   const cx<double>* Y, cx<double>* Rout, double* part, const double* scale) {
  const dim3 grid((unsigned)b.G), blk(WG);
  if (b.groups == kRowsQuads)
    k_defect<kRowsQuads><<<grid, blk, 0, s>>>(b, sigma_col, F, Y, Rout, part, scale);
  else if (b.groups == kRowsTriples)
    k_defect<kRowsTriples><<<grid, blk, 0, s>>>(b, sigma_col, F, Y, Rout, part, scale);
  else
    k_defect<kRowsGeneric><<<grid, blk, 0, s>>>(b, sigma_col, F, Y, Rout, part, scale);
}

// scale_c = ||R_c|| unless the defect meets its target; the next FP32 solve of
// the column only has to reduce R_c by the remaining factor target ||F|| / ||R||,
// so its tolerance is a tenth of that, within [min32, 1e-1].
__global__ __launch_bounds__(WG) void k_defect_norms(Batch b, const double* __restrict__ part,
                                                    const double* __restrict__ tol, int first,
                                                    double* __restrict__ fnorm, double* __restrict__ scale,
                                                    double* __restrict__ relres, float* __restrict__ tol32,
                                                    double min32) {
  constexpr int V = kMixedV;
  SC_PROLOGUE(V)
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const int c = cg0 + v;
    const bool ok = cl0 + v < I.K;
    // a column that met its target keeps its values (its Y no longer changes)
    const bool fresh = ok && (first || scale[c] > 0);
    const double r = sqrt(block_col_sum(part, b.G, I.rot, b.Ktot, c, fresh));
    if (!lead || cl0 + v >= I.Kp || (ok && !fresh)) continue;
    if (first) fnorm[c] = r;
    const double fn = fnorm[c];
    const bool done = !ok || r <= tol[c] * fn;
    scale[c] = done ? 0.0 : r;
    relres[c] = fn > 0 ? r / fn : 0.0;
    const double gap = r > 0 ? tol[c] * fn / r : 1.0;
    tol32[c] = (float)fmin(1e-1, fmax(min32, 0.1 * gap));
  }
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

// r = R / scale (R null: F / scale), rhat = r, x = 0 in FP32; partial |r|^2
__global__ __launch_bounds__(WG) void k_mixed_rhs(Batch b, const cx<double>* __restrict__ R,
                                                 const double* __restrict__ F, const double* __restrict__ scale,
                                                 KrylovState<float> st, cx<float>* __restrict__ rhat) {
  constexpr int V = kMixedV;
  const WgPos p = wg_pos(b.G);
  FOR_TILES(b, p, V)
    float nn[V] = {};
    const bool open = valid && tile_open<V>(scale, cg0, cl0, I.K);
    if (valid && !open && b.sgs) {
      // multicolour SGS recomputes the start values of every tile from r: a tile
      // whose columns all met their targets starts from r = 0, x = 0 (elsewhere
      // its columns simply start converged and keep their old vectors)
      FOR_ROWS(b, p, I)
        const size_t e = tb + (size_t)pos * (WAVE * V);
        const cvec<float, V> z{};
        stv<float, V>(st.r + e, z);
        stv<float, V>(st.x + e, z);
      END_ROWS
    }
    if (open) {
      double inv[V];
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const double sc = scale[cg0 + v];
        inv[v] = (cl0 + v < I.K && sc > 0) ? 1.0 / sc : 0.0;
      }
      FOR_ROWS(b, p, I)
        const int i = pos;
        const size_t e = tb + (size_t)i * (WAVE * V);
        cvec<float, V> r, x;
#pragma unroll
        for (int v = 0; v < V; ++v) {
          const cx<double> d = R ? R[e + v] : cx<double>{F[I.rl + (size_t)i * I.L + col_rhs(cc0 + v, I.L, I.N, I.rmaj)], 0.0};
          r.c[v] = {(float)(d.re * inv[v]), (float)(d.im * inv[v])};
          x.c[v] = {0.f, 0.f};
          // explicit fused steps: the F and the R copies round |r|^2 alike
          nn[v] = fmaf(r.c[v].re, r.c[v].re, fmaf(r.c[v].im, r.c[v].im, nn[v]));
        }
        stv<float, V>(st.r + e, r);
        stv<float, V>(rhat + e, r);
        stv<float, V>(st.x + e, x);
      END_ROWS
    }
    wg_store_partial<float, V>(nn, p.w, p.lane, cl0, I.K, st.part_b + po);
  }
}

void launch_mixed_rhs(hipStream_t s, const Batch& b, const cx<double>* R, const double* F, const double* scale,
                      const KrylovState<float>& st, cx<float>* rhat) {
  k_mixed_rhs<<<dim3((unsigned)b.G), dim3(WG), 0, s>>>(b, R, F, scale, st, rhat);
}

// Y += scale x (first: Y = scale x)
__global__ __launch_bounds__(WG) void k_accumulate(Batch b, const cx<float>* __restrict__ x,
                                                  const double* __restrict__ scale, cx<double>* __restrict__ Y,
                                                  int first) {
  constexpr int V = kMixedV;
  const WgPos p = wg_pos(b.G);
  FOR_TILES(b, p, V)
    (void)po;
    if (!valid || (!first && !tile_open<V>(scale, cg0, cl0, I.K))) continue;
    double sc[V];
#pragma unroll
    for (int v = 0; v < V; ++v) sc[v] = cl0 + v < I.K ? scale[cg0 + v] : 0.0;
    FOR_ROWS(b, p, I)
      const size_t e = tb + (size_t)pos * (WAVE * V);
      const cvec<float, V> xv = ldv<float, V>(x + e);
#pragma unroll
      for (int v = 0; v < V; ++v) {
        if (sc[v] > 0) {
          cx<double> y = first ? cx<double>{0.0, 0.0} : Y[e + v];
          y.re += sc[v] * (double)xv.c[v].re;
          y.im += sc[v] * (double)xv.c[v].im;
          Y[e + v] = y;
        } else if (first) {
          Y[e + v] = {0.0, 0.0};
        }
      }
    END_ROWS
  }
}

void launch_accumulate(hipStream_t s, const Batch& b, const cx<float>* x, const double* scale, cx<double>* Y,
                       int first) {
  k_accumulate<<<dim3((unsigned)b.G), dim3(WG), 0, s>>>(b, x, scale, Y, first);
}

// ---- COCG (conjugate orthogonal CG) for the complex-symmetric shifted systems ----
// S = A - sigma B is complex symmetric, so CG with the bilinear form [u, v] = u^T v
// applies (van der Vorst and Melissen 1990): one sparse product per iteration.
// Point Jacobi (M = diag(S)) or node block Jacobi (M = the 3x3 node blocks of S,
// complex symmetric; the vector kernels then walk nodes); z = M^{-1} r is never
// stored.
// Storage: p in ph (the gathered direction), q = S p in v.
//   start:  p = M^{-1} r, rho = [r, p]           (after k_init / k_mixed_rhs)
//   q = S p, alpha = rho / [p, q]
//   x += alpha p, r -= alpha q                    -> stop if ||r|| <= tol ||f||
//   rho' = [r, M^{-1} r], beta = rho' / rho, p = M^{-1} r + beta p

// Node block Jacobi inside the COCG kernels: z = M_k^{-1} r for node k (rows
// 3k .. 3k + 2) of the lane's columns; M_k^{-1} is the (pole, node) 3x3 inverse
// (row-major, complex symmetric).  Columns past K take z = 0.
template <typename R, int V>
__device__ __forceinline__ void node_apply(const Inst& I, int k, int cl0, int cc0, const cvec<R, V> (&r)[3],
                                           cvec<R, V> (&z)[3]) {
  const int nodes = I.n / 3;
#pragma unroll
  for (int v = 0; v < V; ++v) {
    if (cl0 + v >= I.K) {
#pragma unroll
      for (int i = 0; i < 3; ++i) z[i].c[v] = {0, 0};
      continue;
    }
    const cx<R>* m = static_cast<const cx<R>*>(I.bjac) + ((size_t)col_pole(cc0 + v, I.L, I.N, I.rmaj) * nodes + (size_t)k) * 9;
#pragma unroll
    for (int i = 0; i < 3; ++i)
      z[i].c[v] = cadd(cadd(cmul(m[3 * i], r[0].c[v]), cmul(m[3 * i + 1], r[1].c[v])), cmul(m[3 * i + 2], r[2].c[v]));
  }
}

// p = M^{-1} r over every tile; partial [r, p] in part_a
template <typename R>
__global__ __launch_bounds__(WG, 4) void k_cocg_start(Batch b, KrylovState<R> st) {
  constexpr int V = LaneWidth<R>::V;
  const WgPos p = wg_pos(b.G);
  FOR_TILES(b, p, V)
    cx<R> rz[V] = {};
    if (valid && I.bjac) {  // node block Jacobi: one node (three rows) per wavefront step
      for (int k = blockIdx.x * 4 + p.w; k < I.n / 3; k += b.G * 4) {
        const size_t e0 = tb + (size_t)(3 * k) * (WAVE * V);
        cvec<R, V> r[3], z[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) r[i] = ldv<R, V>(st.r + e0 + (size_t)i * (WAVE * V));
        node_apply<R, V>(I, k, cl0, cc0, r, z);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
#pragma unroll
          for (int v = 0; v < V; ++v) {
            const cx<R> t = cmul(r[i].c[v], z[i].c[v]);
            rz[v].re += t.re;
            rz[v].im += t.im;
          }
          stv<R, V>(st.ph + e0 + (size_t)i * (WAVE * V), z[i]);
        }
      }
    } else if (valid) {
      int pole[V];
#pragma unroll
      for (int v = 0; v < V; ++v) pole[v] = col_pole(cc0 + v, I.L, I.N, I.rmaj);
      FOR_ROWS(b, p, I)
        const size_t e = tb + (size_t)pos * (WAVE * V);
        const size_t de = I.dn + (size_t)pos * I.N;
        const cvec<R, V> r = ldv<R, V>(st.r + e);
        cvec<R, V> z;
#pragma unroll
        for (int v = 0; v < V; ++v) {
          z.c[v] = cl0 + v < I.K ? cmul(st.dinv[de + pole[v]], r.c[v]) : cx<R>{0, 0};
          const cx<R> t = cmul(r.c[v], z.c[v]);
          rz[v].re += t.re;
          rz[v].im += t.im;
        }
        stv<R, V>(st.ph + e, z);
      END_ROWS
    }
    wg_store_partial_cx<R, V>(rz, p.w, p.lane, cl0, I.K, st.part_a + po);
  }
}

// start values: ||f|| from part_b (written by the right-hand-side kernel), rho
// from part_a; every tile starts on the active list, padding columns converged
template <typename R>
__global__ __launch_bounds__(kScWG) void k_cocg_init_scalars(Batch b, KrylovState<R> st) {
  constexpr int V = LaneWidth<R>::V;
  SC_PROLOGUE(V)
  if (threadIdx.x == 0) {
    b.active[blockIdx.x] = blockIdx.x;
    if (blockIdx.x == 0) b.n_active[0] = b.n_tiles;
  }
  // with SGS both sums come from the first forward sweep
  const SlotSet live = I.sgs ? sweep_shares(I, b) : SlotSet{};
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const int c = cg0 + v;
    const bool ok = cl0 + v < I.K;
    const R nn = block_col_sum(st.part_b, b.G, I.rot, b.Ktot, c, ok, live);
    const cx<R> rz = block_col_sum_cx(st.part_a, b.G, I.rot, b.Ktot, c, ok, live);
    if (!lead || cl0 + v >= I.Kp) continue;
    st.fnorm[c] = sqrt(nn);
    st.rnorm[c] = sqrt(nn);
    st.rho[c] = rz;
    st.alpha[c] = {0, 0};
    st.beta[c] = {0, 0};
    st.iters[c] = 0;
    st.flags[c] = (nn == 0 || !ok) ? COL_CONVERGED : COL_ACTIVE;
  }
}

// q = S p; partial [p, q]
template <typename R, int MODE>
__global__ __launch_bounds__(WG, 4) void k_cocg_spmm(Batch b, KrylovState<R> st, int* counter) {
  constexpr int V = LaneWidth<R>::V;
  const WgPos p = wg_pos(b.G);
  FOR_ACTIVE_TILES(b, p, V)
    cx<R> d[V] = {};
    if (tile_has<V>(st.flags, cg0, cl0, I.K, COL_ACTIVE, COL_ACTIVE)) {
      count_tile(counter);
      cx<R> sig[V];
#pragma unroll
      for (int v = 0; v < V; ++v) sig[v] = st.sigma_col[cg0 + v];
      spmm_rows<R, V, MODE>(b, p, I, I.ab, st.ph + tb, sig, [&](int i, const cvec<R, V>& q) {
        if (!valid) return;
        const size_t e = tb + (size_t)i * (WAVE * V);
        stv_nt<R, V>(st.v + e, q);
        const cvec<R, V> pv = ldv<R, V>(st.ph + e);
#pragma unroll
        for (int v = 0; v < V; ++v) {
          const cx<R> t = cmul(pv.c[v], q.c[v]);
          d[v].re += t.re;
          d[v].im += t.im;
        }
      });
    }
    wg_store_partial_cx<R, V>(d, p.w, p.lane, cl0, I.K, st.part_a + po);
  }
}

// alpha = rho / [p, q]
template <typename R>
__global__ __launch_bounds__(kScWG) void k_cocg_alpha(Batch b, KrylovState<R> st) {
  constexpr int V = LaneWidth<R>::V;
  SC_PROLOGUE(V)
  if (!tile_has<V>(st.flags, cg0, cl0, I.K, COL_ACTIVE, COL_ACTIVE)) return;
  // [p, q] from the forward sweeps (SGS) or from the row blocks of the product
  const SlotSet live = I.sgs ? sweep_shares(I, b) : rows_live(I);
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const int c = cg0 + v;
    const bool ok = cl0 + v < I.K;
    const cx<R> pq = block_col_sum_cx(st.part_a, b.G, I.rot, b.Ktot, c, ok, live);
    if (!lead || !ok || st.flags[c] != COL_ACTIVE) continue;
    const cx<R> rho = st.rho[c];
    if ((pq.re == 0 && pq.im == 0) || (rho.re == 0 && rho.im == 0) || !cfinite(pq)) {
      st.flags[c] = COL_BREAKDOWN;
      continue;
    }
    st.alpha[c] = cdiv(rho, pq);
    st.iters[c] += 1;
  }
}

// x += alpha p, r -= alpha q for active columns; partials [r, M^{-1} r] and ||r||^2.
// A pure stream: non-temporal loads and stores.
template <typename R>
__global__ __launch_bounds__(WG, 4) void k_cocg_update_xr(Batch b, KrylovState<R> st, int* counter) {
  constexpr int V = LaneWidth<R>::V;
  const WgPos p = wg_pos(b.G);
  FOR_ACTIVE_TILES(b, p, V)
    const bool node_rows = I.bjac && !I.sgs;
    if (node_rows ? (int)blockIdx.x * 4 >= I.n / 3 : step_block(I, p, 0) < 0) {  // no rows here
      if (counter && tile_has<V>(st.flags, cg0, cl0, I.K, COL_ACTIVE, COL_ACTIVE)) count_tile(counter);
      zero_partial_cx<R, V>(p.w, p.lane, cl0, I.K, st.part_a + po);
      zero_partial<R, V>(p.w, p.lane, cl0, I.K, st.part_b + po);
      continue;
    }
    cx<R> rz[V] = {};
    R nn[V] = {};
    if (tile_has<V>(st.flags, cg0, cl0, I.K, COL_ACTIVE, COL_ACTIVE)) {
      count_tile(counter);
      int f[V], pole[V];
      lane_flags<V>(st.flags, cg0, cl0, I.K, f);
      cx<R> alpha[V];
#pragma unroll
      for (int v = 0; v < V; ++v) {
        pole[v] = col_pole(cc0 + v, I.L, I.N, I.rmaj);
        alpha[v] = f[v] == COL_ACTIVE ? st.alpha[cg0 + v] : cx<R>{0, 0};
      }
      if (node_rows) {  // node block Jacobi: one node per wavefront step
        for (int k = blockIdx.x * 4 + p.w; k < I.n / 3; k += b.G * 4) {
          const size_t e0 = tb + (size_t)(3 * k) * (WAVE * V);
          cvec<R, V> x[3], r[3], pv[3], q[3], z[3];
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            const size_t e = e0 + (size_t)i * (WAVE * V);
            x[i] = ldv_nt<R, V>(st.x + e);
            r[i] = ldv_nt<R, V>(st.r + e);
            pv[i] = ldv_nt<R, V>(st.ph + e);
            q[i] = ldv_nt<R, V>(st.v + e);
          }
#pragma unroll
          for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int v = 0; v < V; ++v) {
              if (f[v] != COL_ACTIVE) continue;
              x[i].c[v] = cadd(x[i].c[v], cmul(alpha[v], pv[i].c[v]));
              r[i].c[v] = csub(r[i].c[v], cmul(alpha[v], q[i].c[v]));
            }
          node_apply<R, V>(I, k, cl0, cc0, r, z);
#pragma unroll
          for (int i = 0; i < 3; ++i) {
#pragma unroll
            for (int v = 0; v < V; ++v) {
              if (f[v] != COL_ACTIVE) continue;
              const cx<R> rv = r[i].c[v];
              const cx<R> t = cmul(rv, z[i].c[v]);
              rz[v].re += t.re;
              rz[v].im += t.im;
              nn[v] += rv.re * rv.re + rv.im * rv.im;
            }
            stv_nt<R, V>(st.x + e0 + (size_t)i * (WAVE * V), x[i]);
            stv_nt<R, V>(st.r + e0 + (size_t)i * (WAVE * V), r[i]);
          }
        }
      } else {
      constexpr int kRowBatch = 2;
      FOR_ROW_BATCH(b, p, I, kRowBatch)
        size_t e[kRowBatch];
        cvec<R, V> x[kRowBatch], r[kRowBatch], pv[kRowBatch], q[kRowBatch];
#pragma unroll
        for (int u = 0; u < kRowBatch; ++u) {
          e[u] = tb + (size_t)ic[u] * (WAVE * V);
          x[u] = ldv_nt<R, V>(st.x + e[u]);
          r[u] = ldv_nt<R, V>(st.r + e[u]);
          pv[u] = ldv_nt<R, V>(st.ph + e[u]);
          q[u] = ldv_nt<R, V>(st.v + e[u]);
        }
#pragma unroll
        for (int u = 0; u < kRowBatch; ++u) {
          if (!ok[u]) continue;
          const size_t de = I.dn + (size_t)ic[u] * I.N;
#pragma unroll
          for (int v = 0; v < V; ++v) {
            if (f[v] != COL_ACTIVE) continue;
            x[u].c[v] = cadd(x[u].c[v], cmul(alpha[v], pv[u].c[v]));
            const cx<R> rv = csub(r[u].c[v], cmul(alpha[v], q[u].c[v]));
            r[u].c[v] = rv;
            // split system of the multicolour SGS: no further preconditioner, [r, r]
            const cx<R> t = I.sgs ? cmul(rv, rv) : cmul(rv, cmul(st.dinv[de + pole[v]], rv));
            rz[v].re += t.re;
            rz[v].im += t.im;
            nn[v] += rv.re * rv.re + rv.im * rv.im;
          }
          stv_nt<R, V>(st.x + e[u], x[u]);
          stv_nt<R, V>(st.r + e[u], r[u]);
        }
      END_ROWS
      }
    }
    wg_store_partial_cx<R, V>(rz, p.w, p.lane, cl0, I.K, st.part_a + po);
    wg_store_partial<R, V>(nn, p.w, p.lane, cl0, I.K, st.part_b + po);
  }
}

// ||r|| test; beta = rho' / rho
template <typename R>
__global__ __launch_bounds__(kScWG) void k_cocg_beta(Batch b, KrylovState<R> st, R tol, int maxit) {
  constexpr int V = LaneWidth<R>::V;
  SC_PROLOGUE(V)
  if (!tile_has<V>(st.flags, cg0, cl0, I.K, COL_ACTIVE, COL_ACTIVE)) return;
  // sums of the x, r update: row blocks, or grid-strided nodes (node block Jacobi)
  const SlotSet live = I.bjac && !I.sgs ? SlotSet{} : rows_live(I);
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const int c = cg0 + v;
    const bool ok = cl0 + v < I.K;
    const cx<R> rz = block_col_sum_cx(st.part_a, b.G, I.rot, b.Ktot, c, ok, live);
    const R nn = sqrt(block_col_sum(st.part_b, b.G, I.rot, b.Ktot, c, ok, live));
    if (!lead || !ok || st.flags[c] != COL_ACTIVE) continue;
    st.rnorm[c] = nn;
    if (nn <= (st.tolc ? st.tolc[c] : tol) * st.fnorm[c]) {
      st.flags[c] = COL_CONVERGED;
      continue;
    }
    if (st.iters[c] >= maxit) {
      st.flags[c] = COL_MAXIT;
      continue;
    }
    if (!cfinite(rz)) {
      st.flags[c] = COL_BREAKDOWN;
      continue;
    }
    st.beta[c] = cdiv(rz, st.rho[c]);
    st.rho[c] = rz;
  }
}

// p = M^{-1} r + beta p for active columns
template <typename R>
__global__ __launch_bounds__(WG, 4) void k_cocg_update_p(Batch b, KrylovState<R> st, int* counter) {
  constexpr int V = LaneWidth<R>::V;
  const WgPos p = wg_pos(b.G);
  FOR_ACTIVE_TILES(b, p, V)
    (void)po;
    if (!tile_has<V>(st.flags, cg0, cl0, I.K, COL_ACTIVE, COL_ACTIVE)) continue;
    count_tile(counter);
    int f[V], pole[V];
    lane_flags<V>(st.flags, cg0, cl0, I.K, f);
    cx<R> beta[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      pole[v] = col_pole(cc0 + v, I.L, I.N, I.rmaj);
      beta[v] = st.beta[cg0 + v];
    }
    if (I.bjac) {  // node block Jacobi: one node per wavefront step
      for (int k = blockIdx.x * 4 + p.w; k < I.n / 3; k += b.G * 4) {
        const size_t e0 = tb + (size_t)(3 * k) * (WAVE * V);
        cvec<R, V> r[3], pv[3], z[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          r[i] = ldv<R, V>(st.r + e0 + (size_t)i * (WAVE * V));
          pv[i] = ldv<R, V>(st.ph + e0 + (size_t)i * (WAVE * V));
        }
        node_apply<R, V>(I, k, cl0, cc0, r, z);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
#pragma unroll
          for (int v = 0; v < V; ++v)
            if (f[v] == COL_ACTIVE) pv[i].c[v] = cadd(z[i].c[v], cmul(beta[v], pv[i].c[v]));
          stv<R, V>(st.ph + e0 + (size_t)i * (WAVE * V), pv[i]);
        }
      }
      continue;
    }
    constexpr int kRowBatch = 4;
    FOR_ROW_BATCH(b, p, I, kRowBatch)
      size_t e[kRowBatch];
      cvec<R, V> r[kRowBatch], pv[kRowBatch];
#pragma unroll
      for (int u = 0; u < kRowBatch; ++u) {
        e[u] = tb + (size_t)ic[u] * (WAVE * V);
        r[u] = ldv<R, V>(st.r + e[u]);
        pv[u] = ldv<R, V>(st.ph + e[u]);
      }
#pragma unroll
      for (int u = 0; u < kRowBatch; ++u) {
        if (!ok[u]) continue;
        const size_t de = I.dn + (size_t)ic[u] * I.N;
#pragma unroll
        for (int v = 0; v < V; ++v) {
          if (f[v] != COL_ACTIVE) continue;
          pv[u].c[v] = cadd(cmul(st.dinv[de + pole[v]], r[u].c[v]), cmul(beta[v], pv[u].c[v]));
        }
        stv<R, V>(st.ph + e[u], pv[u]);
      }
    END_ROWS
  }
}

// ---- multicolour symmetric Gauss-Seidel, split (Eisenstat) form ---------------
//
// M = (D + L) D^{-1} (D + U) with D the point or node blocks of S = A - sigma B
// and L / U its couplings to nodes of lower / higher colour.  With D = R R^T
// (complex symmetric factor) M = M_L M_L^T, M_L = (D + L) R^{-T}, and COCG runs
// on W y' = M_L^{-1} f with W = M_L^{-1} S M_L^{-T} (complex symmetric).  Since
// S = (D + L) + (D + U) - D,
//   W p = R^T (t + u),  t = (D + U)^{-1} R p,  u = (D + L)^{-1} (R p - D t),
// one backward and one forward sweep: each touches every coupling once, so an
// iteration reads the pattern once, as one product with S would.  A sweep runs
// one launch per colour (the nodes of a colour are not coupled); node k of
// colour c gathers t (backward) or u (forward) of the already finished colours.
//   start:  u = (D + L)^{-1} f, r' = R^T u, rho = [r', r'], ||f'|| = ||r'||
//   iteration: p = r' + beta p (first: p = r'), backward and forward sweeps give
//           q = W p and [p, q]; alpha; x' += alpha p, r' -= alpha q; beta
//   finish: y = (D + U)^{-1} R x'
// The partial sums of the forward sweeps are accumulated over the colour
// launches in the workgroup's slot (fixed order: bitwise reproducible).  A
// node's own rows are read and written once per launch and go through
// non-temporal accesses: L2 is left to the gathered rows of its neighbours.
constexpr int kSgsBackIter = 0, kSgsBackFinal = 1, kSgsFwdIter = 2, kSgsFwdStart = 3;

template <typename T, int V>
__device__ __forceinline__ void wg_acc_partial(const T (&v)[V], int w, int lane, int cl0, int K, T* out, bool add) {
  __shared__ T red[4][V * WAVE];
#pragma unroll
  for (int u = 0; u < V; ++u) red[w][V * lane + u] = v[u];
  __syncthreads();
  if (w == 0) {
#pragma unroll
    for (int u = 0; u < V; ++u) {
      const int k = V * lane + u;
      if (cl0 + u < K) out[k] = (add ? out[k] : T(0)) + (red[0][k] + red[1][k] + red[2][k] + red[3][k]);
    }
  }
  __syncthreads();
}

template <typename R, int V>
__device__ __forceinline__ void wg_acc_partial_cx(const cx<R> (&v)[V], int w, int lane, int cl0, int K, cx<R>* out,
                                                  bool add) {
  R re[V], im[V];
#pragma unroll
  for (int u = 0; u < V; ++u) {
    re[u] = v[u].re;
    im[u] = v[u].im;
  }
  __shared__ R rr[4][V * WAVE], ri[4][V * WAVE];
#pragma unroll
  for (int u = 0; u < V; ++u) {
    rr[w][V * lane + u] = re[u];
    ri[w][V * lane + u] = im[u];
  }
  __syncthreads();
  if (w == 0) {
#pragma unroll
    for (int u = 0; u < V; ++u) {
      const int k = V * lane + u;
      if (cl0 + u < K) {
        const cx<R> o = add ? out[k] : cx<R>{0, 0};
        out[k] = {o.re + (rr[0][k] + rr[1][k] + rr[2][k] + rr[3][k]), o.im + (ri[0][k] + ri[1][k] + ri[2][k] + ri[3][k])};
      }
    }
  }
  __syncthreads();
}

// y_i = sum_j m_ij x_j (TR: m_ji) for a BS x BS block of one column
template <typename R, int BS, bool TR>
__device__ __forceinline__ void blk_apply(const cx<R>* __restrict__ m, const cx<R> (&x)[BS], cx<R> (&y)[BS]) {
#pragma unroll
  for (int i = 0; i < BS; ++i) {
    cx<R> acc{0, 0};
#pragma unroll
    for (int j = 0; j < BS; ++j) acc = cadd(acc, cmul(m[TR ? BS * j + i : BS * i + j], x[j]));
    y[i] = acc;
  }
}

// The couplings of node k's rows to the other colours' nodes, applied to the
// gathered block G (the lower or the upper CSR): acc_r = sum_j S_{row r, j} G_j.
template <typename R, int V, int BS>
__device__ __forceinline__ void sgs_couplings(const Inst& I, int k, const int* rp, const int* cl, const void* abv,
                                              const cx<R>* __restrict__ Gc, const cx<R> (&sig)[V],
                                              cvec<R, V> (&acc)[BS]) {
  const cptr<int> rowptr = as_const(rp), col = as_const(cl);
  const cptr<ab_pair<R>> ab = as_const(static_cast<const ab_pair<R>*>(abv));
  if constexpr (BS == 3) {
    if (I.nodes && as_const(I.nodes)[k] != 0) {
      shifted_node<R, V, true, kSgsNodeChunk>(3 * k, rowptr, col, ab, Gc, WAVE * V, sig, acc);
      return;
    }
#pragma unroll
    for (int r = 0; r < 3; ++r)
      acc[r] = shifted_row<R, V, kChunkShared<R>, true>(3 * k + r, rowptr, col, ab, Gc, WAVE * V, sig);
  } else {
    acc[0] = shifted_row<R, V, kChunk, true>(k, rowptr, col, ab, Gc, WAVE * V, sig);
  }
}

// Per-column diagonal-block data of node k: R, D and D^{-1} for the column's pole.
template <typename R, int BS>
struct SgsBlocks {
  const cx<R>* Rm;
  const cx<R>* Dm;
  const cx<R>* Di;
};

template <typename R, int BS>
__device__ __forceinline__ SgsBlocks<R, BS> sgs_blocks(const Inst& I, const KrylovState<R>& st, int k, int pole) {
  if constexpr (BS == 3) {
    const size_t o = ((size_t)pole * (size_t)(I.n / 3) + (size_t)k) * 9;
    return {static_cast<const cx<R>*>(I.sgsR) + o, static_cast<const cx<R>*>(I.sgsD) + o,
            static_cast<const cx<R>*>(I.bjac) + o};
  } else {
    const size_t o = (size_t)k * I.N + pole;
    return {static_cast<const cx<R>*>(I.sgsR) + o, st.d + I.dn + o, st.dinv + I.dn + o};
  }
}

template <typename R, int BS, int MODE>
__global__ __launch_bounds__(WG, 4) void k_sgs_sweep(Batch b, KrylovState<R> st, int colour, int add, int first,
                                                     int* counter) {
  constexpr int V = LaneWidth<R>::V;
  constexpr bool all_tiles = MODE == kSgsBackFinal || MODE == kSgsFwdStart;
  constexpr bool fwd = MODE == kSgsFwdIter || MODE == kSgsFwdStart;
  const WgPos p = wg_pos(b.Gs);
  FOR_TILE_LIST(b, p, V, all_tiles ? b.n_tiles : as_const((const int*)b.n_active)[0],
                all_tiles ? ti_ : as_const((const int*)b.active)[ti_])
    if (I.sgs != BS) continue;  // the other block size's launch owns this pencil's tiles
    // share g = x * per + q of the colour's nodes: sgs_share consecutive nodes
    // (a multiple of 4: each wavefront takes the same number), XCD by XCD
    int q0 = 0, q1 = 0;
    if (colour < I.sgs_ncol) {
      const cptr<int> cptr_ = as_const(I.sgs_cptr);
      const int c0 = cptr_[colour], c1 = cptr_[colour + 1];
      q0 = c0 + (p.x * p.per + p.q) * I.sgs_share;
      q1 = min(c1, q0 + I.sgs_share);
    }
    if (q0 >= q1) {  // no nodes here: zero partials, written by the first colour launch
      if (counter && colour < I.sgs_ncol &&
          (all_tiles || tile_has<V>(st.flags, cg0, cl0, I.K, COL_ACTIVE, COL_ACTIVE)))
        count_tile(counter);
      if (fwd && !add) {
        zero_partial_cx<R, V>(p.w, p.lane, cl0, I.K, st.part_a + po);
        if (MODE == kSgsFwdStart) zero_partial<R, V>(p.w, p.lane, cl0, I.K, st.part_b + po);
      }
      continue;
    }
    cx<R> da[V] = {};
    R db[V] = {};
    const bool go = all_tiles || tile_has<V>(st.flags, cg0, cl0, I.K, COL_ACTIVE, COL_ACTIVE);
    if (go) {
      count_tile(counter);
      int f[V], pole[V];
      cx<R> sig[V], beta[V];
      lane_flags<V>(st.flags, cg0, cl0, I.K, f);
#pragma unroll
      for (int v = 0; v < V; ++v) {
        pole[v] = col_pole(cc0 + v, I.L, I.N, I.rmaj);
        sig[v] = st.sigma_col[cg0 + v];
        beta[v] = st.beta[cg0 + v];
      }
      const cptr<int> nodes = as_const(I.sgs_nodes);
      for (int q = q0 + p.w; q < q1; q += 4) {
        const int k = nodes[q];
        const size_t e0 = tb + (size_t)(BS * k) * (WAVE * V);
        cvec<R, V> own[BS], two[BS], acc[BS];
        // own: the vector the sweep transforms; two: t (forward iteration)
#pragma unroll
        for (int i = 0; i < BS; ++i) {
          const size_t e = e0 + (size_t)i * (WAVE * V);
          if (MODE == kSgsBackIter) {
            const cvec<R, V> rv = ldv_nt<R, V>(st.r + e);
            cvec<R, V> pv = first ? rv : ldv_nt<R, V>(st.ph + e);
            if (!first) {
#pragma unroll
              for (int v = 0; v < V; ++v)
                if (f[v] == COL_ACTIVE) pv.c[v] = cadd(rv.c[v], cmul(beta[v], pv.c[v]));
            }
            own[i] = pv;
          } else if (MODE == kSgsBackFinal) {
            own[i] = ldv_nt<R, V>(st.x + e);
          } else if (MODE == kSgsFwdIter) {
            own[i] = ldv_nt<R, V>(st.ph + e);
            two[i] = ldv_nt<R, V>(st.t + e);
          } else {
            own[i] = ldv_nt<R, V>(st.r + e);
          }
        }
        if (fwd)
          sgs_couplings<R, V, BS>(I, k, I.lrp, I.lcol, I.lab, st.sh + tb, sig, acc);
        else
          sgs_couplings<R, V, BS>(I, k, I.urp, I.ucol, I.uab, st.t + tb, sig, acc);
        cvec<R, V> res[BS], out2[BS];
#pragma unroll
        for (int v = 0; v < V; ++v) {
          const SgsBlocks<R, BS> m = sgs_blocks<R, BS>(I, st, k, pole[v]);
          cx<R> x[BS], w[BS], y[BS];
#pragma unroll
          for (int i = 0; i < BS; ++i) x[i] = own[i].c[v];
          if (MODE == kSgsFwdStart) {
#pragma unroll
            for (int i = 0; i < BS; ++i) w[i] = x[i];
          } else {
            blk_apply<R, BS, false>(m.Rm, x, w);  // R p (R x')
          }
          if (MODE == kSgsFwdIter) {
            cx<R> tv[BS], dt[BS];
#pragma unroll
            for (int i = 0; i < BS; ++i) tv[i] = two[i].c[v];
            blk_apply<R, BS, false>(m.Dm, tv, dt);
#pragma unroll
            for (int i = 0; i < BS; ++i) w[i] = csub(w[i], dt[i]);
          }
#pragma unroll
          for (int i = 0; i < BS; ++i) w[i] = csub(w[i], acc[i].c[v]);
          blk_apply<R, BS, false>(m.Di, w, y);  // t or u
#pragma unroll
          for (int i = 0; i < BS; ++i) res[i].c[v] = y[i];
          if (MODE == kSgsFwdIter || MODE == kSgsFwdStart) {
            cx<R> z[BS], o[BS];
#pragma unroll
            for (int i = 0; i < BS; ++i) z[i] = MODE == kSgsFwdIter ? cadd(two[i].c[v], y[i]) : y[i];
            blk_apply<R, BS, true>(m.Rm, z, o);  // R^T (t + u) or R^T u
#pragma unroll
            for (int i = 0; i < BS; ++i) {
              out2[i].c[v] = o[i];
              if (cl0 + v < I.K) {
                const cx<R> a = MODE == kSgsFwdIter ? x[i] : o[i];
                const cx<R> pq = cmul(a, o[i]);
                da[v].re += pq.re;
                da[v].im += pq.im;
                if (MODE == kSgsFwdStart) db[v] += o[i].re * o[i].re + o[i].im * o[i].im;
              }
            }
          }
        }
        if (!valid) continue;
#pragma unroll
        for (int i = 0; i < BS; ++i) {
          const size_t e = e0 + (size_t)i * (WAVE * V);
          if (MODE == kSgsBackIter) {
            stv_nt<R, V>(st.ph + e, own[i]);
            stv_nt<R, V>(st.t + e, res[i]);
          } else if (MODE == kSgsBackFinal) {
            stv_nt<R, V>(st.t + e, res[i]);
            stv_nt<R, V>(st.x + e, res[i]);
          } else if (MODE == kSgsFwdIter) {
            stv_nt<R, V>(st.sh + e, res[i]);
            stv_nt<R, V>(st.v + e, out2[i]);
          } else {
            stv_nt<R, V>(st.sh + e, res[i]);
            stv_nt<R, V>(st.r + e, out2[i]);
          }
        }
      }
    }
    if (fwd) {
      wg_acc_partial_cx<R, V>(da, p.w, p.lane, cl0, I.K, st.part_a + po, add != 0);
      if (MODE == kSgsFwdStart) wg_acc_partial<R, V>(db, p.w, p.lane, cl0, I.K, st.part_b + po, add != 0);
    }
  }
}

template <typename R, int BS, int MODE>
void sgs_sweeps(hipStream_t s, const Batch& b, const KrylovState<R>& st, int first, LaunchTimer* tm,
                double tile_bytes, double fixed) {
  const dim3 grid((unsigned)b.Gs), blk(WG);
  constexpr bool fwd = MODE == kSgsFwdIter || MODE == kSgsFwdStart;
  const int nc = b.sgs_ncol;
  for (int q = 0; q < nc; ++q) {
    const int c = fwd ? q : nc - 1 - q;
    // a colour launch of one direction does 1 / (2 nc) of a product with S
    int* cnt = tm ? tm->begin(s, 0, tile_bytes / nc, fixed / nc, 0.5 / nc, b.Gs) : nullptr;
    k_sgs_sweep<R, BS, MODE><<<grid, blk, 0, s>>>(b, st, c, q > 0 ? 1 : 0, first, cnt);
    if (cnt) tm->end(s);
  }
}

// One COCG iteration on the split system: the backward colour sweeps of every
// block size present in the batch (each launch serves the pencils of its block
// size), then the forward ones, then the scalars and the x, r update.
template <typename R>
void sgs_iteration(hipStream_t s, const Batch& b, const KrylovState<R>& st, R tol, int maxit, bool first,
                   LaunchTimer* tm, const IterBytes& by) {
  const dim3 grid((unsigned)b.G), blk(WG);
  const dim3 cgrid((unsigned)b.n_tiles), cblk(kScWG);
  // backward: read r, p; write p, t; gather t once; the upper couplings and the blocks
  const double tb = 5 * by.blk + 0.5 * by.sgs_blocks;
  if (b.sgs & 1) sgs_sweeps<R, 1, kSgsBackIter>(s, b, st, first ? 1 : 0, tm, tb, by.sgs_upper);
  if (b.sgs & 2) sgs_sweeps<R, 3, kSgsBackIter>(s, b, st, first ? 1 : 0, tm, tb, by.sgs_upper);
  // forward: read p, t; write u, q; gather u once; the lower couplings and the blocks
  if (b.sgs & 1) sgs_sweeps<R, 1, kSgsFwdIter>(s, b, st, 0, tm, tb, by.sgs_lower);
  if (b.sgs & 2) sgs_sweeps<R, 3, kSgsFwdIter>(s, b, st, 0, tm, tb, by.sgs_lower);
  k_cocg_alpha<R><<<cgrid, cblk, 0, s>>>(b, st);
  int* c = tm ? tm->begin(s, 1, 6 * by.blk, 0) : nullptr;
  k_cocg_update_xr<R><<<grid, blk, 0, s>>>(b, st, c);
  if (c) tm->end(s);
  k_cocg_beta<R><<<cgrid, cblk, 0, s>>>(b, st, tol, maxit);
}

template <typename R>
void launch_sgs_finish(hipStream_t s, const Batch& b, const KrylovState<R>& st) {
  if (b.sgs & 1) sgs_sweeps<R, 1, kSgsBackFinal>(s, b, st, 0, nullptr, 0, 0);
  if (b.sgs & 2) sgs_sweeps<R, 3, kSgsBackFinal>(s, b, st, 0, nullptr, 0, 0);
}

template <typename R>
void launch_cocg_start(hipStream_t s, const Batch& b, const KrylovState<R>& st) {
  if (b.sgs) {
    if (b.sgs & 1) sgs_sweeps<R, 1, kSgsFwdStart>(s, b, st, 0, nullptr, 0, 0);
    if (b.sgs & 2) sgs_sweeps<R, 3, kSgsFwdStart>(s, b, st, 0, nullptr, 0, 0);
  } else {
    k_cocg_start<R><<<dim3((unsigned)b.G), dim3(WG), 0, s>>>(b, st);
  }
  k_cocg_init_scalars<R><<<dim3((unsigned)b.n_tiles), dim3(kScWG), 0, s>>>(b, st);
}

template <typename R>
void launch_cocg_iteration(hipStream_t s, const Batch& b, const KrylovState<R>& st, R tol, int maxit,
                           bool first, LaunchTimer* tm, const IterBytes& by) {
  if (b.sgs) {
    sgs_iteration<R>(s, b, st, tol, maxit, first, tm, by);
    return;
  }
  const dim3 grid((unsigned)b.G), blk(WG);
  const dim3 cgrid((unsigned)b.n_tiles), cblk(kScWG);
  int* c;
  // q = S p: gather p once, write q, read p's own rows; the merged CSR once
  c = tm ? tm->begin(s, 0, 2 * by.blk, by.matrix) : nullptr;
  if (b.groups == kRowsQuads)
    k_cocg_spmm<R, kRowsQuads><<<grid, blk, 0, s>>>(b, st, c);
  else if (b.groups == kRowsTriples)
    k_cocg_spmm<R, kRowsTriples><<<grid, blk, 0, s>>>(b, st, c);
  else
    k_cocg_spmm<R, kRowsGeneric><<<grid, blk, 0, s>>>(b, st, c);
  if (c) tm->end(s);
  k_cocg_alpha<R><<<cgrid, cblk, 0, s>>>(b, st);
  // x, r update: read x, r, p, q, write x, r; 1/d
  c = tm ? tm->begin(s, 1, 6 * by.blk + by.diag, 0) : nullptr;
  k_cocg_update_xr<R><<<grid, blk, 0, s>>>(b, st, c);
  if (c) tm->end(s);
  k_cocg_beta<R><<<cgrid, cblk, 0, s>>>(b, st, tol, maxit);
  // p update: read r, p, write p; 1/d
  c = tm ? tm->begin(s, 1, 3 * by.blk + by.diag, 0) : nullptr;
  k_cocg_update_p<R><<<grid, blk, 0, s>>>(b, st, c);
  if (c) tm->end(s);
}

#define SLRF_INST(R)                                                                                  \
  template void launch_init<R>(hipStream_t, const Batch&, const KrylovState<R>&, const R*);        \
  template void launch_init_scalars<R>(hipStream_t, const Batch&, const KrylovState<R>&);          \
  template void launch_iteration<R>(hipStream_t, const Batch&, const KrylovState<R>&, R, int, bool, \
                                    int, LaunchTimer*, const IterBytes&);                              \
  template void launch_cocg_start<R>(hipStream_t, const Batch&, const KrylovState<R>&);            \
  template void launch_cocg_iteration<R>(hipStream_t, const Batch&, const KrylovState<R>&, R, int, \
                                         bool, LaunchTimer*, const IterBytes&);                         \
  template void launch_sgs_finish<R>(hipStream_t, const Batch&, const KrylovState<R>&);
SLRF_INST(double)
SLRF_INST(float)

}  // namespace slrf

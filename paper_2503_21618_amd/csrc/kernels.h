// Device-side data types and kernel launchers of the SLRF library (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace slrf {

template <typename R>
struct alignas(2 * sizeof(R)) cx {
  R re, im;
};

// One merged-CSR value: stiffness a_ij and mass b_ij of the same entry.
template <typename R>
struct alignas(2 * sizeof(R)) ab_pair {
  R a, b;
};

// Per-column state of the inner BiCGStab solves.
enum ColFlag : int {
  COL_ACTIVE = 0,
  COL_CONVERGED = 1,
  COL_HALF_CONVERGED = 2,
  COL_BREAKDOWN = 3,
  COL_MAXIT = 4,
  COL_HALF_PENDING = 5,  // converged at the half step; x still takes alpha * p_hat
};

constexpr int kMaxGrid = 2048;  // largest grid of the Krylov kernels (a multiple of 8)
constexpr int kCsrPad = 16;     // zero entries after the last CSR entry (whole-chunk reads)

// One pencil of a batch as the Krylov kernels see it.  Its Krylov block is a
// row-major (n, Kp) complex array, K = N * L, column c = j * L + l belonging to
// pole j and right-hand side l (columns K..Kp-1 are padding).  Global columns of
// the batch are the pencils' Kp columns one after the other; global tiles of
// 64 V columns likewise.
struct Inst {
  int n, K, L, N;        // rows, columns, right-hand sides, poles
  int Kp;                // padded columns: K rounded up to a whole tile (blocks are tile-major)
  int nrb, slab, steps;  // row blocks, row blocks per XCD, steps per workgroup
  int rot;               // rotation of the pencil's row blocks over an XCD's workgroups
  int rmaj;              // column order: 0 pole-major, 1 right-hand-side-major (col_pole)
  int col0, tile0;       // first global column and first global tile
  int nnz;
  int64_t blk;           // element offset of the (n, K) blocks
  int64_t rl;            // element offset of the (n, L) real blocks (rhat, F)
  int64_t dn;            // element offset of the (n, N) diagonal blocks
  const int* rowptr;
  const int* col;
  const void* ab;               // ab_pair<R> in the Krylov precision
  const ab_pair<double>* ab64;  // FP64 values (defect of the mixed path)
  const int* sched;             // sparse-product row order, or null
  const int* groups;            // stencil-group flags per kGroup rows, or null
  const int* nodes;             // node-triple flags per 3 rows, or null
  const int* diagpos;           // position of each row's diagonal (ILU)
  const void* ilu;              // (N, nnz) cx<R> ILU(0) factors, or null
  const void* bjac;             // (N, n/3, 3, 3) cx<R> inverted node blocks, or null
  // Multicolour symmetric Gauss-Seidel (COCG only): sgs = block size (1 point, 3
  // node blocks) or 0.  Nodes of colour c are sgs_nodes[sgs_cptr[c] .. sgs_cptr[c+1]);
  // the couplings of each row to nodes of lower (l*) and higher (u*) colours form
  // two CSR matrices with (a, b) pairs in the Krylov precision.  sgsR holds R with
  // D = R R^T for each pole's diagonal block D of A - sigma B (point: (n, N) at
  // Inst::dn like d; blocks: (N, n/3, 3, 3) row-major), sgsD the node blocks D
  // (blocks only; point pencils use d), bjac their inverses (blocks; point: dinv).
  int sgs, sgs_ncol;
  int sgs_share, sgs_wgs;  // nodes of a colour per sweep workgroup (a multiple of 4), shares used
  const int* sgs_cptr;
  const int* sgs_nodes;
  const int* lrp;
  const int* lcol;
  const void* lab;
  const int* urp;
  const int* ucol;
  const void* uab;
  const void* sgsR;
  const void* sgsD;
};

// Column order of a pencil's blocks.  Pole-major (rmaj = 0): column c = j L + l
// holds right-hand side l (column l of B X) for pole j, so a tile belongs to
// one pole and the tiles of fast poles retire early.  Right-hand-side-major
// (rmaj = 1, used with warm starts): c = l N + j, so a tile covers a few
// right-hand sides for every pole and right-hand sides that start close to
// their solutions retire whole tiles.  Padding columns (c >= N L) map to the
// last pole and right-hand side.
__host__ __device__ inline int col_pole(int c, int L, int N, int rmaj) {
  return rmaj ? c % N : (c / L < N ? c / L : N - 1);
}
__host__ __device__ inline int col_rhs(int c, int L, int N, int rmaj) {
  return rmaj ? (c / N < L ? c / N : L - 1) : c % L;
}
__host__ __device__ inline int col_of(int j, int l, int L, int N, int rmaj) { return rmaj ? l * N + j : j * L + l; }

// Kernel argument describing a whole batch (device tables).
struct Batch {
  const Inst* inst;       // [count]
  const int* tile_inst;   // [n_tiles] pencil of each global tile
  const int* col_inst;    // [Ktot] pencil of each global column
  int* active;            // [n_tiles] tiles that had an active column at the last poll
  int* n_active;          // [1] length of that list
  int n_tiles;
  int Ktot;               // global columns, each pencil padded to Kp
  int G;                  // grid, a multiple of 8
  int Gs;                 // grid of the multicolour SGS sweeps, a multiple of 8
  int rows_per_block;
  int V;                  // columns per lane (1 for complex FP64, 2 for complex FP32)
  int groups;             // sparse-product row mode: 1 stencil groups, 2 node triples, 0 neither
  int sgs;                // multicolour SGS of the batch's pencils: bit 0 point, bit 1 node blocks
  int sgs_ncol;           // most colours of any pencil (sweeps launch once per colour)
};

// Krylov vectors: base pointers of the concatenated per-pencil blocks; per
// column arrays are indexed by global column; partial sums are [G][Ktot].
template <typename R>
struct KrylovState {
  cx<R>* x;
  cx<R>* r;
  cx<R>* ph;   // preconditioned search direction M^{-1} p
  cx<R>* v;
  cx<R>* sh;   // preconditioned half-step residual M^{-1} s
  cx<R>* t;
  cx<R>* p;    // unpreconditioned search direction (general preconditioner only)
  cx<R>* s;    // unpreconditioned half-step residual (general preconditioner only)
  const R* rhat;         // real (n, L) shadow residual per pencil (at Inst::rl)
  const cx<R>* rhat_cx;  // per-column complex shadow residual (at Inst::blk), if non-null
  const cx<R>* d;        // (n, N) shifted-operator diagonals (at Inst::dn)
  const cx<R>* dinv;
  const cx<R>* sigma_col;  // [Ktot] pole of each column
  const R* tolc;           // [Ktot] relative tolerance of each column, or null (one for all)
  cx<R>* part_a;
  R* part_b;
  cx<R>* rho;
  cx<R>* alpha;
  cx<R>* omega;
  cx<R>* beta;
  R* fnorm;
  R* rnorm;
  int* flags;
  int* iters;
};

// Optional per-launch instrumentation of the Krylov kernels: a HIP event pair
// around each sparse-product / vector-update launch and a device counter of the
// (workgroup, tile) pairs the launch processed (tiles whose columns are all
// converged exit at once).
struct LaunchTimer {
  hipEvent_t* events = nullptr;  // 2 * capacity
  int* d_counts = nullptr;       // capacity
  int capacity = 0;
  int used = 0;
  struct Rec {
    int kind;           // 0 sparse product, 1 vector update
    double tile_bytes;  // bytes of a launch that processes every tile (scale with tiles)
    double fixed;       // bytes read once per launch whatever the tiles (merged CSR)
    double share;       // share of one product with S a full-width launch performs
    int grid;           // workgroups of the launch (0: the batch grid G)
  };
  Rec recs[512];
  int* begin(hipStream_t s, int kind, double tile_bytes, double fixed, double share = 1.0, int grid = 0);
  void end(hipStream_t s);
};

// Algorithmic byte counts of one batch iteration (for the timer).
struct IterBytes {
  double blk;      // one pass over every (n, K) block
  double rhat;     // the (n, L) real blocks
  double diag;     // the (n, N) diagonal blocks
  double matrix;   // every merged CSR once
  double sgs_lower, sgs_upper;  // the lower / upper coupling CSRs once (multicolour SGS)
  double sgs_blocks;            // R, D and D^{-1} of every pole once (multicolour SGS)
};

// ---- batched Krylov launchers (stream-ordered) ----------------------------
template <typename R>
void launch_init(hipStream_t s, const Batch& b, const KrylovState<R>& st, const R* F);
template <typename R>
void launch_init_scalars(hipStream_t s, const Batch& b, const KrylovState<R>& st);
template <typename R>
// precs: 1 if some pencil uses ILU(0), 2 if some pencil uses node block Jacobi (or both)
void launch_iteration(hipStream_t s, const Batch& b, const KrylovState<R>& st, R tol, int maxit,
                      bool first, int precs, LaunchTimer* timer, const IterBytes& bytes);
// COCG (point Jacobi only): p = M^{-1} r and the per-column start values, after
// launch_init or launch_mixed_rhs has written r and the partial ||r||^2; then
// one COCG iteration per call.
template <typename R>
void launch_cocg_start(hipStream_t s, const Batch& b, const KrylovState<R>& st);
template <typename R>
void launch_cocg_iteration(hipStream_t s, const Batch& b, const KrylovState<R>& st, R tol, int maxit,
                           bool first, LaunchTimer* timer, const IterBytes& bytes);
// Batches with multicolour SGS (Batch::sgs) run COCG on the split system
// W y' = f', W = M_L^{-1} S M_L^{-T}, M_L = (D + L) R^{-T}, f' = M_L^{-1} f: the
// start transforms r = f into f' (forward colour sweeps), each iteration forms
// q = W p by one backward and one forward sweep (Eisenstat: no separate product
// with S), and launch_sgs_finish turns x = y' into y = M_L^{-T} y' (backward
// sweeps) for every column.
template <typename R>
void launch_sgs_finish(hipStream_t s, const Batch& b, const KrylovState<R>& st);
// out[0] = number of active columns; rebuilds the active-tile list of the batch.
void launch_count_active(hipStream_t s, const Batch& b, const int* flags, int* out);

// Mixed precision (FP32 inner solves, FP64 defect correction).
// R = F - S Y in FP64 (Y null: R = F and R is not written), partial |R|^2 in part [G][Ktot].
// With Y, tiles whose columns all have scale 0 (met their target earlier) are skipped.
void launch_defect(hipStream_t s, const Batch& b, const cx<double>* sigma_col, const double* F,
                   const cx<double>* Y, cx<double>* Rout, double* part, const double* scale);
// scale_c = ||R_c|| if ||R_c|| > tol_c ||F_c|| else 0 (tol per column); the first round
// sets fnorm_c = ||F_c||; tol32_c = clamp(0.1 tol_c ||F_c|| / ||R_c||, min32, 0.1), the
// relative tolerance of the column's next FP32 solve; *count = columns with scale_c > 0.
void launch_defect_norms(hipStream_t s, const Batch& b, const double* part, const double* tol,
                         int first, double* fnorm, double* scale, double* relres, float* tol32,
                         double min32, int* count);
// r = R / scale (R null: F / scale), rhat = r, x = 0 in FP32; partial |r|^2 into part_b.
void launch_mixed_rhs(hipStream_t s, const Batch& b, const cx<double>* R, const double* F,
                      const double* scale, const KrylovState<float>& st, cx<float>* rhat);
// Y += scale x (first: Y = scale x)
void launch_accumulate(hipStream_t s, const Batch& b, const cx<float>* x, const double* scale,
                       cx<double>* Y, int first);

// ---- per-pencil launchers -------------------------------------------------
template <typename R>
void launch_jacobi_diag(hipStream_t s, int n, int N, const R* diagA, const R* diagB,
                        const cx<R>* sigma, cx<R>* d, cx<R>* dinv, double cd = 1.0, double ci = 1.0);
// U = sum_j 2 Re(w_j x[:, j L .. j L + L)), x a tile-major block (tiles of W
// columns, each an n x W row-major panel)
template <typename R>
void launch_filter_sum(hipStream_t s, int n, int L, int N, int W, int rmaj, const cx<R>* x,
                       const double* w /* 2N */, double* U, bool accumulate);

// Y0 = Y_prev C per pole (C real L x L row-major), tile-major complex FP64
// blocks with tiles of W columns and Kp padded columns (padding set to zero)
void launch_recycle(hipStream_t s, int n, int L, int N, int W, int Kp, int rmaj, const cx<double>* Yp,
                    const double* C, cx<double>* Y0);

// real products with the merged pencil: AX = A X, BX = B X (either may be null)
template <typename R>
void launch_spmm_real(hipStream_t s, int n, int L, const int* rowptr, const int* col,
                      const ab_pair<R>* ab, const double* X, double* AX, double* BX);

// Gram matrices GA = U^T WA, GB = U^T WB (L x L), FP64 MFMA (f32: FP32 MFMA on
// the inputs rounded to FP32, FP32 accumulation), deterministic.
void launch_gram(hipStream_t s, int n, int L, const double* U, const double* WA,
                 const double* WB, double* part, int nchunks, double* GA, double* GB, bool f32 = false);
int gram_chunks(int n, int L);

// Y_b = X_b Z for b < nb blocks (n x L times L x r), FP64 MFMA.
void launch_gemm_nz(hipStream_t s, int n, int L, int r, int nb, const double* const* X,
                    const double* Z, double* const* Y);

// per-column sums of |AX - theta BX|^2 and |BX|^2 over row blocks of 256
void launch_resid(hipStream_t s, int n, int L, const double* AX, const double* BX,
                  const double* theta, double* part /* [nrb][2][L] */, int nrb);

void launch_gaussian(hipStream_t s, int64_t count, uint64_t seed, double* out);
void launch_fill_zero(hipStream_t s, void* p, size_t bytes);

}  // namespace slrf

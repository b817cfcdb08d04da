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

// Geometry of an (n, K) complex Krylov block: rows split into row blocks of
// `rows_per_block`, columns into tiles of 64 (one column per lane).  Every
// kernel over the block uses the same grid of G workgroups, so per-column
// partial sums live in [G][K] arrays and are reduced in a fixed order.
struct KGeom {
  int n;
  int K;             // columns = poles * L, pole-major (c = j * L + l)
  int L;
  int N;             // poles
  int rows_per_block;
  int nrb;           // row blocks
  int nct;           // column tiles of 64
  int slab;          // row blocks per XCD
  int G;             // workgroups (a multiple of 8)
  int steps;         // row-block steps per tile per workgroup
  const int* sched;  // sparse-product row order (a permutation of 0..n-1), or null
};
constexpr int kMaxGrid = 1024;  // G <= kMaxGrid

KGeom make_geom(int n, int N, int L, int rows_per_block);

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
  const R* rhat;       // (n, L) shared shadow residual = right-hand side
  const cx<R>* rhat_cx;  // (n, K) per-column complex shadow residual (used when non-null)
  const cx<R>* d;      // (n, N) shifted-operator diagonal
  const cx<R>* dinv;   // (n, N) its inverse
  const cx<R>* sigma_col;  // (K) pole of each column
  cx<R>* part_a;       // (nrb, K) complex partial sums
  R* part_b;           // (nrb, K) real partial sums
  // per-column scalars
  cx<R>* rho;
  cx<R>* alpha;
  cx<R>* omega;
  cx<R>* beta;
  R* fnorm;
  R* rnorm;
  int* flags;
  int* iters;
};

// ILU(0) factors of A - sigma_j B on the merged pattern, one value array per pole
// (L strictly lower with unit diagonal, U upper; the U diagonal is stored inverted).
template <typename R>
struct IluFactors {
  const int* rowptr;
  const int* col;
  const int* diagpos;  // position of the diagonal entry in each row
  const cx<R>* f;      // (N, nnz)
  int64_t nnz;
};

// Optional per-launch instrumentation of the Krylov kernels: a HIP event pair
// around each sparse-product / vector-update launch and a device counter of the
// column tiles the launch processed (tiles whose columns are all converged exit
// at once).  Host-side records say which kernel and how many n x K passes it
// makes per processed tile.
struct LaunchTimer {
  hipEvent_t* events = nullptr;  // 2 * capacity
  int* d_counts = nullptr;       // capacity
  int capacity = 0;
  int used = 0;
  struct Rec {
    int kind;           // 0 sparse product, 1 vector update
    double tile_bytes;  // bytes of a launch that processes every tile (scale with tiles)
    double fixed;       // bytes read once per launch whatever the tiles (merged CSR)
  };
  Rec recs[512];
  // returns the counter for the next launch (records its start event) or nullptr
  int* begin(hipStream_t s, int kind, double tile_bytes, double fixed);
  void end(hipStream_t s);
};

// ---- launchers (stream-ordered) -----------------------------------------
template <typename R>
void launch_jacobi_diag(hipStream_t s, int n, int N, const R* diagA, const R* diagB,
                        const cx<R>* sigma, cx<R>* d, cx<R>* dinv);
template <typename R>
void launch_init(hipStream_t s, const KGeom& g, const KrylovState<R>& st, const R* F);
template <typename R>
void launch_init_scalars(hipStream_t s, const KGeom& g, const KrylovState<R>& st);
template <typename R>
void launch_iteration(hipStream_t s, const KGeom& g, const KrylovState<R>& st,
                      const int* rowptr, const int* col, const ab_pair<R>* ab,
                      R tol, int maxit, bool first, const IluFactors<R>* ilu,
                      LaunchTimer* timer, double matrix_bytes);
void launch_count_active(hipStream_t s, int K, const int* flags, int* out);

// ---- mixed precision (FP32 inner solves, FP64 defect correction) ----------
// R = F - S Y over all K columns in FP64 (Y null: R = F, R not written), with
// per-column partial sums of |R|^2 into part [G][K].
void launch_defect(hipStream_t s, const KGeom& g, const int* rowptr, const int* col,
                   const ab_pair<double>* ab, const cx<double>* sigma_col, const double* F,
                   const cx<double>* Y, cx<double>* Rout, double* part);
// scale_c = ||R_c|| if ||R_c|| > tol ||F_c|| else 0; fnorm_c = ||F_c|| on the first
// round (first != 0); writes the number of unconverged columns to *count.
void launch_defect_norms(hipStream_t s, const KGeom& g, const double* part, double tol, int first,
                         double* fnorm, double* scale, double* relres, int* count);
// r = R / scale (R null: F / scale), rhat = r, x = 0 in FP32; partial |r|^2 into part_b.
void launch_mixed_rhs(hipStream_t s, const KGeom& g, const cx<double>* R, const double* F,
                      const double* scale, const KrylovState<float>& st, cx<float>* rhat);
// Y += scale x (first: Y = scale x)
void launch_accumulate(hipStream_t s, const KGeom& g, const cx<float>* x, const double* scale,
                       cx<double>* Y, int first);

template <typename R>
void launch_filter_sum(hipStream_t s, int n, int L, int N, const cx<R>* x,
                       const double* w /* 2N */, double* U, bool accumulate);

// real products with the merged pencil: AX = A X, BX = B X (either may be null)
template <typename R>
void launch_spmm_real(hipStream_t s, int n, int L, const int* rowptr, const int* col,
                      const ab_pair<R>* ab, const double* X, double* AX, double* BX);

// Gram matrices GA = U^T WA, GB = U^T WB (L x L), FP64 MFMA, deterministic.
void launch_gram(hipStream_t s, int n, int L, const double* U, const double* WA,
                 const double* WB, double* part, int nchunks, double* GA, double* GB);
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

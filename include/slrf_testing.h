/*
 * slrf_testing.h -- kernel-level test hooks of libslrf (not part of the solver
 * API).  They run single internal kernels so that tests can compare them element
 * by element with a CPU reference.  All pointers are DEVICE pointers, row-major,
 * float64; work is enqueued on hip_stream (NULL = default) and synchronised.
 * Return 0 on success, SLRF_E_INVALID_ARG / SLRF_E_DEVICE otherwise.
 */
#ifndef SLRF_TESTING_H
#define SLRF_TESTING_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

/* GA = U^T WA and GB = U^T WB for U, WA, WB of shape (n, L); GA, GB (L, L).
 * The Gram step of the Rayleigh-Ritz projection (Algorithm 1, forming the
 * projected pencil), FP64 MFMA with a deterministic split over rows. */
int slrf_test_gram(int64_t n, int64_t L, const double* U, const double* WA, const double* WB,
                   double* GA, double* GB, void* scratch, size_t scratch_bytes, void* hip_stream);

/* Y = X Z for X (n, L), Z (L, r), Y (n, r): the Ritz-vector update x_i = U s_i
 * (Algorithm 1), FP64 MFMA. */
int slrf_test_gemm(int64_t n, int64_t L, int64_t r, const double* X, const double* Z, double* Y,
                   void* hip_stream);

/* The Gram products with a choice of arithmetic: f32 = 0 FP64 MFMA
 * (v_mfma_f64_16x16x4), f32 = 1 FP32 MFMA (v_mfma_f32_16x16x4, inputs rounded to
 * FP32, FP32 accumulation), the first projection of a mixed-precision outer
 * iteration while its Ritz pairs are far from converged. */
int slrf_test_gram_prec(int64_t n, int64_t L, const double* U, const double* WA, const double* WB,
                        double* GA, double* GB, void* scratch, size_t scratch_bytes, int f32,
                        void* hip_stream);

/* Bytes of scratch slrf_test_gram needs. */
size_t slrf_test_gram_scratch(int64_t n, int64_t L);

#ifdef __cplusplus
}
#endif
#endif

/*
 * lddmm_alg3.h -- C ABI of liblddmm_alg3, the materialised-matrix forward
 * step (paper Sec. 2.4, Alg. 3) rebuilt on MI355X as a measured ablation.
 *
 * The paper's first GPU design computes every pair term of one forward step
 * (eq. 2) into N x N matrices in device memory and sums each row with a BLAS
 * matrix-vector product against a vector of ones; Sec. 2.4 names its two
 * costs, N^2 storage and an N^2 write and re-read through global memory.
 * This library reproduces that design with a HIP kernel for the terms and
 * rocBLAS sgemv for the sums, so that its time and memory can be set beside
 * the fused pair kernels of liblddmm.  It is context only: liblddmm's calls
 * do not use it.
 *
 * Computed (FP32 terms, FP32 sums, FP64 in and out), for every landmark i:
 *   Hp_i = sum_j g_ij p_j,   Hq_i = -(1/sigma^2) sum_j g_ij (p_i . p_j)(q_i - q_j),
 *   g_ij = exp(-|q_i - q_j|^2 / (2 sigma^2)), j = i included,
 * i.e. (dH/dp, dH/dq) of eq. 2 with H = 1/2 <p, K(q) p>.  The six term
 * matrices are stored [6][N][N] (component, i, j; j contiguous): 24 N^2
 * bytes of workspace (403 MB at N = 4096).
 */
#ifndef LDDMM_ALG3_H
#define LDDMM_ALG3_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lddmm_alg3 lddmm_alg3;

/* Status codes: 0 ok, -1 invalid argument, -2 device allocation failed,
 * -3 HIP or rocBLAS error (detail from lddmm_alg3_last_error). */

/* Binds `device` and creates the rocBLAS handle.  *out receives the context. */
int lddmm_alg3_create(int device, lddmm_alg3** out);

/* Frees the handle and the context; NULL is accepted. */
int lddmm_alg3_destroy(lddmm_alg3* ctx);

/* Workspace bytes one call with n landmarks needs: the six N x N FP32 term
 * matrices, the 6 N row sums and a vector of N ones (each 256-byte aligned). */
size_t lddmm_alg3_workspace_bytes(int32_t n);

/* One forward step's pair sums by Alg. 3 (Sec. 2.4).
 *   n          : landmarks, 1..16384
 *   sigma      : Gaussian kernel width, > 0
 *   q, p       : in,  [n][3] device FP64 (landmark state q_t, p_t)
 *   hq, hp     : out, [n][3] device FP64, dH/dq and dH/dp
 *   ws         : device workspace of ws_bytes >= lddmm_alg3_workspace_bytes(n),
 *                or NULL to allocate it and free it inside the call, as the
 *                paper's listing does (MemAlloc before, cudaFree after)
 *   stream     : hipStream_t as void* (NULL: the null stream); with ws == NULL
 *                the call waits for the stream before freeing
 * Returns 0, or a negative status before anything is enqueued for invalid
 * arguments. */
int lddmm_alg3_pair_forward(lddmm_alg3* ctx, int32_t n, double sigma, const double* q,
                            const double* p, double* hq, double* hp, void* ws, size_t ws_bytes,
                            void* stream);

/* Detail of the last error on ctx (or of the last call without one). */
const char* lddmm_alg3_last_error(lddmm_alg3* ctx);

#ifdef __cplusplus
}
#endif

#endif /* LDDMM_ALG3_H */

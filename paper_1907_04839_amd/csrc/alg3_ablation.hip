// The materialised-matrix forward step of the paper's Sec. 2.4 (Alg. 3) on
// gfx950, kept apart from liblddmm as a measured ablation: every pair term of
// eq. 2 is written to device memory (six N x N FP32 matrices) and each row is
// summed by rocBLAS sgemv against a vector of ones.
//
// Launches of one call: a staging kernel (FP32 SoA copies of k q and p, the
// ones vector), the term kernel (one workgroup row of 256 j per i, every
// term written with coalesced stores), one sgemv over the [6N x N] matrix,
// and a kernel that scales and transposes the 6 N sums into the FP64 [n][3]
// outputs.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <new>
#include <string>

#include "lddmm_alg3.h"

struct lddmm_alg3 {
  int device = 0;
  rocblas_handle blas = nullptr;
  std::string err;
};

namespace {

constexpr int kMaxN = 16384;
constexpr int kThreads = 256;

thread_local std::string g_err;

int fail(lddmm_alg3* c, int st, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
int fail(lddmm_alg3* c, int st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  (c ? c->err : g_err) = buf;
  return st;
}

size_t a256(size_t b) { return (b + 255) & ~size_t(255); }

struct Ws {
  float *terms, *sums, *ones, *xs, *ps;
};

Ws carve(void* base, int n) {
  const size_t nn = (size_t)n * n;
  char* b = static_cast<char*>(base);
  Ws w;
  w.terms = reinterpret_cast<float*>(b);
  b += a256(6 * nn * sizeof(float));
  w.sums = reinterpret_cast<float*>(b);
  b += a256(6 * (size_t)n * sizeof(float));
  w.ones = reinterpret_cast<float*>(b);
  b += a256((size_t)n * sizeof(float));
  w.xs = reinterpret_cast<float*>(b);
  b += a256(3 * (size_t)n * sizeof(float));
  w.ps = reinterpret_cast<float*>(b);
  return w;
}

// FP32 SoA copies: xs = k q (so that g = exp2(-|xs_i - xs_j|^2)), ps = p; ones.
__global__ __launch_bounds__(kThreads) void k_alg3_stage(int n, double k,
                                                         const double* __restrict__ q,
                                                         const double* __restrict__ p,
                                                         float* __restrict__ xs,
                                                         float* __restrict__ ps,
                                                         float* __restrict__ ones) {
  const int j = blockIdx.x * kThreads + threadIdx.x;
  if (j >= n) return;
  for (int c = 0; c < 3; ++c) {
    xs[c * n + j] = (float)(k * q[3 * j + c]);
    ps[c * n + j] = (float)p[3 * j + c];
  }
  ones[j] = 1.0f;
}

// Terms of row i (blockIdx.y) for 256 j: T[c][i][j] = g p_j[c] (c < 3) and
// g (p_i . p_j) (k q_i - k q_j)[c - 3] (c >= 3).
__global__ __launch_bounds__(kThreads) void k_alg3_terms(int n, const float* __restrict__ xs,
                                                         const float* __restrict__ ps,
                                                         float* __restrict__ T) {
  const int i = blockIdx.y;
  const int j = blockIdx.x * kThreads + threadIdx.x;
  if (j >= n) return;
  const float xi = xs[i], yi = xs[n + i], zi = xs[2 * n + i];
  const float pxi = ps[i], pyi = ps[n + i], pzi = ps[2 * n + i];
  const float dx = xi - xs[j], dy = yi - xs[n + j], dz = zi - xs[2 * n + j];
  const float pxj = ps[j], pyj = ps[n + j], pzj = ps[2 * n + j];
  const float g = __builtin_amdgcn_exp2f(-(dx * dx + dy * dy + dz * dz));
  const float gs = g * (pxi * pxj + pyi * pyj + pzi * pzj);
  const size_t nn = (size_t)n * n, row = (size_t)i * n + j;
  T[row] = g * pxj;
  T[nn + row] = g * pyj;
  T[2 * nn + row] = g * pzj;
  T[3 * nn + row] = gs * dx;
  T[4 * nn + row] = gs * dy;
  T[5 * nn + row] = gs * dz;
}

// Row sums [6][n] -> hp, hq [n][3] FP64; hq takes the factor -c/k.
__global__ __launch_bounds__(kThreads) void k_alg3_out(int n, double hq_scale,
                                                       const float* __restrict__ sums,
                                                       double* __restrict__ hq,
                                                       double* __restrict__ hp) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  for (int c = 0; c < 3; ++c) {
    hp[3 * i + c] = (double)sums[c * n + i];
    hq[3 * i + c] = hq_scale * (double)sums[(3 + c) * n + i];
  }
}

const char* blas_name(rocblas_status s) { return rocblas_status_to_string(s); }

}  // namespace

extern "C" {

int lddmm_alg3_create(int device, lddmm_alg3** out) {
  if (!out) return fail(nullptr, -1, "out is NULL");
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
    return fail(nullptr, -1, "device %d not available", device);
  if (hipSetDevice(device) != hipSuccess) return fail(nullptr, -3, "hipSetDevice failed");
  lddmm_alg3* c = new (std::nothrow) lddmm_alg3;
  if (!c) return fail(nullptr, -2, "host allocation failed");
  c->device = device;
  const rocblas_status s = rocblas_create_handle(&c->blas);
  if (s != rocblas_status_success) {
    delete c;
    return fail(nullptr, -3, "rocblas_create_handle: %s", blas_name(s));
  }
  *out = c;
  return 0;
}

int lddmm_alg3_destroy(lddmm_alg3* c) {
  if (!c) return 0;
  (void)hipSetDevice(c->device);
  if (c->blas) (void)rocblas_destroy_handle(c->blas);
  delete c;
  return 0;
}

size_t lddmm_alg3_workspace_bytes(int32_t n) {
  if (n < 1) return 0;
  const size_t nn = (size_t)n * n;
  return a256(6 * nn * 4) + a256(6 * (size_t)n * 4) + a256((size_t)n * 4) +
         a256(3 * (size_t)n * 4) + a256(3 * (size_t)n * 4);
}

int lddmm_alg3_pair_forward(lddmm_alg3* c, int32_t n, double sigma, const double* q,
                            const double* p, double* hq, double* hp, void* ws, size_t ws_bytes,
                            void* stream) {
  if (!c) return fail(nullptr, -1, "ctx is NULL");
  if (n < 1 || n > kMaxN) return fail(c, -1, "n must be in 1..%d (got %d)", kMaxN, n);
  if (!(sigma > 0.0) || !std::isfinite(sigma)) return fail(c, -1, "sigma must be finite and > 0");
  if (!q || !p || !hq || !hp) return fail(c, -1, "q, p, hq and hp must not be NULL");
  const size_t need = lddmm_alg3_workspace_bytes(n);
  if (ws && ws_bytes < need)
    return fail(c, -1, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, -3, "hipSetDevice failed");
  hipStream_t s = static_cast<hipStream_t>(stream);
  void* own = nullptr;
  if (!ws) {   // the listing's MemAlloc ... cudaFree around the step
    if (hipMalloc(&own, need) != hipSuccess) {
      (void)hipGetLastError();
      return fail(c, -2, "hipMalloc of %zu bytes failed", need);
    }
    ws = own;
  }
  const Ws w = carve(ws, n);
  const double k = std::sqrt(1.4426950408889634 / (2.0 * sigma * sigma));
  const double hq_scale = -(1.0 / (sigma * sigma)) / k;
  const unsigned blocks = (unsigned)((n + kThreads - 1) / kThreads);
  int st = 0;
  k_alg3_stage<<<blocks, kThreads, 0, s>>>(n, k, q, p, w.xs, w.ps, w.ones);
  k_alg3_terms<<<dim3(blocks, (unsigned)n), kThreads, 0, s>>>(n, w.xs, w.ps, w.terms);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) st = fail(c, -3, "term kernels: %s", hipGetErrorString(e));
  if (st == 0) {
    const float one = 1.0f, zero = 0.0f;
    rocblas_status b = rocblas_set_stream(c->blas, s);
    if (b == rocblas_status_success)
      b = rocblas_sgemv(c->blas, rocblas_operation_transpose, n, 6 * n, &one, w.terms, n, w.ones,
                        1, &zero, w.sums, 1);
    if (b != rocblas_status_success) st = fail(c, -3, "rocblas_sgemv: %s", blas_name(b));
  }
  if (st == 0) {
    k_alg3_out<<<blocks, kThreads, 0, s>>>(n, hq_scale, w.sums, hq, hp);
    e = hipGetLastError();
    if (e != hipSuccess) st = fail(c, -3, "output kernel: %s", hipGetErrorString(e));
  }
  if (own) {
    e = hipStreamSynchronize(s);
    if (e != hipSuccess && st == 0) st = fail(c, -3, "hipStreamSynchronize: %s", hipGetErrorString(e));
    (void)hipFree(own);
  }
  return st;
}

const char* lddmm_alg3_last_error(lddmm_alg3* c) { return c ? c->err.c_str() : g_err.c_str(); }

}  // extern "C"

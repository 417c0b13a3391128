// blas.hip -- FP64 vector kernels of the Krylov solver: block dot products
// (Arnoldi's h_jk = v_j^H w), basis updates, norms, scalings, precision casts.
//
// Reductions are deterministic: each workgroup writes its partial sums, a second
// kernel adds them in a fixed order.  Within a workgroup the sum goes through
// 64-lane wavefront shuffles and one LDS exchange between the four wavefronts.
#include "ddq_internal.h"

namespace ddq {

constexpr int RB = 256;    // threads per reduction workgroup
constexpr int DOT_J = 8;   // basis vectors per dot workgroup

// Basis vectors are streamed once per kernel: non-temporal loads keep them from
// displacing the vector w that the dot kernels re-read per basis chunk.
#ifndef DDQ_BASIS_NT
#define DDQ_BASIS_NT 1
#endif
__device__ __forceinline__ d2_t ld_basis(const d2_t* p) {
#if DDQ_BASIS_NT
  return __builtin_nontemporal_load(p);
#else
  return *p;
#endif
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// sum over the workgroup of NV values per thread; result valid in thread 0 (res[k])
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* lds /* [4][NV] */) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) lds[wave * NV + k] = v[k];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = lds[k] + lds[NV + k] + lds[2 * NV + k] + lds[3 * NV + k];
}

// partial[(j)*nbx + bx] = sum over this workgroup's elements of conj(V_j[e]) w[e],
// j = blockIdx.y * DOT_J + jj
__global__ void __launch_bounds__(RB) k_dot_partial(const d2_t* __restrict__ V, long long vstride, int k,
                                                    const d2_t* __restrict__ w, long long n,
                                                    d2_t* __restrict__ partial) {
  __shared__ double lds[4 * 2 * DOT_J];
  const int j0 = blockIdx.y * DOT_J;
  const int nj = min(DOT_J, k - j0);
  double acc[2 * DOT_J];
#pragma unroll
  for (int q = 0; q < 2 * DOT_J; ++q) acc[q] = 0.0;
  const long long stride = (long long)gridDim.x * RB;
  for (long long e = (long long)blockIdx.x * RB + threadIdx.x; e < n; e += stride) {
    d2_t we = w[e];
#pragma unroll
    for (int jj = 0; jj < DOT_J; ++jj) {
      if (jj < nj) {
        d2_t v = ld_basis(V + (size_t)(j0 + jj) * vstride + e);
        acc[2 * jj] = fma(v.x, we.x, fma(v.y, we.y, acc[2 * jj]));
        acc[2 * jj + 1] = fma(v.x, we.y, fma(-v.y, we.x, acc[2 * jj + 1]));
      }
    }
  }
  block_sum<2 * DOT_J>(acc, lds);
  if (threadIdx.x == 0) {
    for (int jj = 0; jj < nj; ++jj) {
      d2_t o;
      o.x = acc[2 * jj];
      o.y = acc[2 * jj + 1];
      partial[(size_t)(j0 + jj) * gridDim.x + blockIdx.x] = o;
    }
  }
}

hipError_t launch_dot_partial(const d2_t* V, long long vstride, int k, const d2_t* w, long long n,
                              d2_t* partial, int nbx, hipStream_t s) {
  dim3 grid(nbx, (k + DOT_J - 1) / DOT_J);
  hipLaunchKernelGGL(k_dot_partial, grid, dim3(RB), 0, s, V, vstride, k, w, n, partial);
  return hipGetLastError();
}

// out[j] = sum_b partial[j * nbx + b], one workgroup per j
__global__ void __launch_bounds__(RB) k_reduce_partial(const d2_t* __restrict__ partial, int nbx,
                                                       d2_t* __restrict__ out) {
  __shared__ double lds[4 * 2];
  const int j = blockIdx.x;
  double v[2] = {0.0, 0.0};
  for (int b = threadIdx.x; b < nbx; b += RB) {
    d2_t p = partial[(size_t)j * nbx + b];
    v[0] += p.x;
    v[1] += p.y;
  }
  block_sum<2>(v, lds);
  if (threadIdx.x == 0) {
    d2_t o;
    o.x = v[0];
    o.y = v[1];
    out[j] = o;
  }
}

hipError_t launch_reduce_partial(const d2_t* partial, int nbx, int k, d2_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_partial, dim3(k), dim3(RB), 0, s, partial, nbx, out);
  return hipGetLastError();
}

// w[e] += sign * sum_j V_j[e] h[j]
__global__ void __launch_bounds__(RB) k_update(d2_t* __restrict__ w, const d2_t* __restrict__ V,
                                               long long vstride, int k, const d2_t* __restrict__ h,
                                               double sign, long long n) {
  __shared__ d2_t hs[256];
  for (int j = threadIdx.x; j < k; j += RB) hs[j] = h[j];
  __syncthreads();
  const long long stride = (long long)gridDim.x * RB;
  for (long long e = (long long)blockIdx.x * RB + threadIdx.x; e < n; e += stride) {
    double ar = 0.0, ai = 0.0;
    for (int j = 0; j < k; ++j) {
      d2_t v = ld_basis(V + (size_t)j * vstride + e);
      d2_t hj = hs[j];
      ar = fma(v.x, hj.x, fma(-v.y, hj.y, ar));
      ai = fma(v.x, hj.y, fma(v.y, hj.x, ai));
    }
    d2_t we = w[e];
    we.x = fma(sign, ar, we.x);
    we.y = fma(sign, ai, we.y);
    w[e] = we;
    store_fence();
  }
}

static int grid_for(long long n) {
  long long b = (n + RB - 1) / RB;
  return (int)(b > 4096 ? 4096 : (b < 1 ? 1 : b));
}

hipError_t launch_update(d2_t* w, const d2_t* V, long long vstride, int k, const d2_t* h, double sign,
                         long long n, hipStream_t s) {
  if (k > 256) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_update, dim3(grid_for(n)), dim3(RB), 0, s, w, V, vstride, k, h, sign, n);
  return hipGetLastError();
}

__global__ void __launch_bounds__(RB) k_norm2_partial(const d2_t* __restrict__ w, long long n,
                                                      double* __restrict__ partial) {
  __shared__ double lds[4];
  double v[1] = {0.0};
  const long long stride = (long long)gridDim.x * RB;
  for (long long e = (long long)blockIdx.x * RB + threadIdx.x; e < n; e += stride) {
    d2_t a = w[e];
    v[0] = fma(a.x, a.x, fma(a.y, a.y, v[0]));
  }
  block_sum<1>(v, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = v[0];
}

hipError_t launch_norm2_partial(const d2_t* w, long long n, double* partial, int nbx, hipStream_t s) {
  hipLaunchKernelGGL(k_norm2_partial, dim3(nbx), dim3(RB), 0, s, w, n, partial);
  return hipGetLastError();
}

__global__ void __launch_bounds__(RB) k_reduce_real(const double* __restrict__ partial, int nbx,
                                                    double* __restrict__ out) {
  __shared__ double lds[4];
  double v[1] = {0.0};
  for (int b = threadIdx.x; b < nbx; b += RB) v[0] += partial[b];
  block_sum<1>(v, lds);
  if (threadIdx.x == 0) *out = v[0];
}

hipError_t launch_reduce_real(const double* partial, int nbx, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_real, dim3(1), dim3(RB), 0, s, partial, nbx, out);
  return hipGetLastError();
}

__global__ void k_scale(d2_t* __restrict__ out, const d2_t* __restrict__ in, double a, long long n) {
  const long long stride = (long long)gridDim.x * RB;
  for (long long e = (long long)blockIdx.x * RB + threadIdx.x; e < n; e += stride) {
    d2_t v = in[e];
    v.x *= a;
    v.y *= a;
    out[e] = v;
  }
}

hipError_t launch_scale(d2_t* out, const d2_t* in, double a, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_scale, dim3(grid_for(n)), dim3(RB), 0, s, out, in, a, n);
  return hipGetLastError();
}

// out = in / sqrt(*norm2_dev)
__global__ void k_scale_dev(d2_t* __restrict__ out, const d2_t* __restrict__ in, const double* norm2, long long n) {
  const double a = 1.0 / sqrt(*norm2);
  const long long stride = (long long)gridDim.x * RB;
  for (long long e = (long long)blockIdx.x * RB + threadIdx.x; e < n; e += stride) {
    d2_t v = in[e];
    v.x *= a;
    v.y *= a;
    out[e] = v;
  }
}

hipError_t launch_scale_dev(d2_t* out, const d2_t* in, const double* norm2_dev, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_dev, dim3(grid_for(n)), dim3(RB), 0, s, out, in, norm2_dev, n);
  return hipGetLastError();
}

__global__ void k_axpy(d2_t* __restrict__ y, double ar, double ai, const d2_t* __restrict__ x, long long n) {
  const long long stride = (long long)gridDim.x * RB;
  for (long long e = (long long)blockIdx.x * RB + threadIdx.x; e < n; e += stride) {
    d2_t a = x[e], b = y[e];
    b.x = fma(ar, a.x, fma(-ai, a.y, b.x));
    b.y = fma(ar, a.y, fma(ai, a.x, b.y));
    y[e] = b;
  }
}

hipError_t launch_axpy(d2_t* y, double ar, double ai, const d2_t* x, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy, dim3(grid_for(n)), dim3(RB), 0, s, y, ar, ai, x, n);
  return hipGetLastError();
}

__global__ void k_copy(d2_t* __restrict__ y, const d2_t* __restrict__ x, long long n) {
  const long long stride = (long long)gridDim.x * RB;
  for (long long e = (long long)blockIdx.x * RB + threadIdx.x; e < n; e += stride) y[e] = x[e];
}

hipError_t launch_copy(d2_t* y, const d2_t* x, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_copy, dim3(grid_for(n)), dim3(RB), 0, s, y, x, n);
  return hipGetLastError();
}

__global__ void k_scale_f32(f2_t* __restrict__ y, const f2_t* __restrict__ x, float a, long long n) {
  const long long stride = (long long)gridDim.x * RB;
  for (long long e = (long long)blockIdx.x * RB + threadIdx.x; e < n; e += stride) {
    f2_t v = x[e];
    v.x *= a;
    v.y *= a;
    y[e] = v;
  }
}

hipError_t launch_scale_f32(f2_t* y, const f2_t* x, float a, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_f32, dim3(grid_for(n)), dim3(RB), 0, s, y, x, a, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// batched forms: nrhs independent systems, vector r at offset r * n, basis vector
// j of system r at V + j * vstride + r * n
// ---------------------------------------------------------------------------

// partial[(r * k + j) * nbx + bx] = sum over a workgroup's elements of conj(V_j[r]) w[r]
__global__ void __launch_bounds__(RB) k_dot_partial_b(const d2_t* __restrict__ V, long long vstride, int k,
                                                      const d2_t* __restrict__ w, long long n,
                                                      d2_t* __restrict__ partial) {
  __shared__ double lds[4 * 2 * DOT_J];
  const int r = blockIdx.z;
  const int j0 = blockIdx.y * DOT_J;
  const int nj = min(DOT_J, k - j0);
  const d2_t* Vr = V + (size_t)r * n;
  const d2_t* wr = w + (size_t)r * n;
  double acc[2 * DOT_J];
#pragma unroll
  for (int q = 0; q < 2 * DOT_J; ++q) acc[q] = 0.0;
  const long long stride = (long long)gridDim.x * RB;
  for (long long e = (long long)blockIdx.x * RB + threadIdx.x; e < n; e += stride) {
    d2_t we = wr[e];
#pragma unroll
    for (int jj = 0; jj < DOT_J; ++jj) {
      if (jj < nj) {
        d2_t v = ld_basis(Vr + (size_t)(j0 + jj) * vstride + e);
        acc[2 * jj] = fma(v.x, we.x, fma(v.y, we.y, acc[2 * jj]));
        acc[2 * jj + 1] = fma(v.x, we.y, fma(-v.y, we.x, acc[2 * jj + 1]));
      }
    }
  }
  block_sum<2 * DOT_J>(acc, lds);
  if (threadIdx.x == 0) {
    for (int jj = 0; jj < nj; ++jj) {
      d2_t o;
      o.x = acc[2 * jj];
      o.y = acc[2 * jj + 1];
      partial[((size_t)r * k + j0 + jj) * gridDim.x + blockIdx.x] = o;
    }
  }
}

// out[r * ldo + j] = sum_b partial[(r * k + j) * nbx + b]
__global__ void __launch_bounds__(RB) k_reduce_partial_b(const d2_t* __restrict__ partial, int nbx, int k, int ldo,
                                                         d2_t* __restrict__ out) {
  __shared__ double lds[4 * 2];
  const int j = blockIdx.x, r = blockIdx.y;
  double v[2] = {0.0, 0.0};
  const d2_t* p = partial + ((size_t)r * k + j) * nbx;
  for (int b = threadIdx.x; b < nbx; b += RB) {
    d2_t q = p[b];
    v[0] += q.x;
    v[1] += q.y;
  }
  block_sum<2>(v, lds);
  if (threadIdx.x == 0) {
    d2_t o;
    o.x = v[0];
    o.y = v[1];
    out[(size_t)r * ldo + j] = o;
  }
}

hipError_t launch_dot_b(const d2_t* V, long long vstride, int k, const d2_t* w, long long n, int nrhs, d2_t* partial,
                        int nbx, d2_t* out, int ldo, hipStream_t s) {
  if (k < 1) return hipSuccess;
  hipLaunchKernelGGL(k_dot_partial_b, dim3(nbx, (k + DOT_J - 1) / DOT_J, nrhs), dim3(RB), 0, s, V, vstride, k, w, n,
                     partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_partial_b, dim3(k, nrhs), dim3(RB), 0, s, partial, nbx, k, ldo, out);
  return hipGetLastError();
}

// w[r] += sign * sum_{j < k} V_j[r] h[r * ldh + j]
__global__ void __launch_bounds__(RB) k_update_b(d2_t* __restrict__ w, const d2_t* __restrict__ V, long long vstride,
                                                 int k, const d2_t* __restrict__ h, int ldh, double sign, long long n) {
  __shared__ d2_t hs[256];
  const int r = blockIdx.y;
  for (int j = threadIdx.x; j < k; j += RB) hs[j] = h[(size_t)r * ldh + j];
  __syncthreads();
  const d2_t* Vr = V + (size_t)r * n;
  d2_t* wr = w + (size_t)r * n;
  const long long stride = (long long)gridDim.x * RB;
  for (long long e = (long long)blockIdx.x * RB + threadIdx.x; e < n; e += stride) {
    double ar = 0.0, ai = 0.0;
    for (int j = 0; j < k; ++j) {
      d2_t v = ld_basis(Vr + (size_t)j * vstride + e);
      d2_t hj = hs[j];
      ar = fma(v.x, hj.x, fma(-v.y, hj.y, ar));
      ai = fma(v.x, hj.y, fma(v.y, hj.x, ai));
    }
    d2_t we = wr[e];
    we.x = fma(sign, ar, we.x);
    we.y = fma(sign, ai, we.y);
    wr[e] = we;
    store_fence();
  }
}

hipError_t launch_update_b(d2_t* w, const d2_t* V, long long vstride, int k, const d2_t* h, int ldh, double sign,
                           long long n, int nrhs, hipStream_t s) {
  if (k < 1) return hipSuccess;
  if (k > 256) return hipErrorInvalidValue;
  long long b = (n + RB - 1) / RB;
  const int nb = (int)(b > 2048 ? 2048 : b);
  hipLaunchKernelGGL(k_update_b, dim3(nb, nrhs), dim3(RB), 0, s, w, V, vstride, k, h, ldh, sign, n);
  return hipGetLastError();
}

// out[r] = |w[r]|^2
__global__ void __launch_bounds__(RB) k_norm2_partial_b(const d2_t* __restrict__ w, long long n,
                                                        double* __restrict__ partial) {
  __shared__ double lds[4];
  const int r = blockIdx.y;
  const d2_t* wr = w + (size_t)r * n;
  double v[1] = {0.0};
  const long long stride = (long long)gridDim.x * RB;
  for (long long e = (long long)blockIdx.x * RB + threadIdx.x; e < n; e += stride) {
    d2_t a = wr[e];
    v[0] = fma(a.x, a.x, fma(a.y, a.y, v[0]));
  }
  block_sum<1>(v, lds);
  if (threadIdx.x == 0) partial[(size_t)r * gridDim.x + blockIdx.x] = v[0];
}

__global__ void __launch_bounds__(RB) k_reduce_real_b(const double* __restrict__ partial, int nbx,
                                                      double* __restrict__ out) {
  __shared__ double lds[4];
  const int r = blockIdx.x;
  double v[1] = {0.0};
  for (int b = threadIdx.x; b < nbx; b += RB) v[0] += partial[(size_t)r * nbx + b];
  block_sum<1>(v, lds);
  if (threadIdx.x == 0) out[r] = v[0];
}

hipError_t launch_norm2_b(const d2_t* w, long long n, int nrhs, double* partial, int nbx, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_norm2_partial_b, dim3(nbx, nrhs), dim3(RB), 0, s, w, n, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_real_b, dim3(nrhs), dim3(RB), 0, s, partial, nbx, out);
  return hipGetLastError();
}

// out[r] = f[r] * in[r]  (f on the device)
__global__ void k_scale_b(d2_t* __restrict__ out, const d2_t* __restrict__ in, const double* __restrict__ f,
                          long long n) {
  const int r = blockIdx.y;
  const double a = f[r];
  const long long stride = (long long)gridDim.x * RB;
  for (long long e = (long long)blockIdx.x * RB + threadIdx.x; e < n; e += stride) {
    d2_t v = in[(size_t)r * n + e];
    v.x *= a;
    v.y *= a;
    out[(size_t)r * n + e] = v;
  }
}

hipError_t launch_scale_b(d2_t* out, const d2_t* in, const double* f, long long n, int nrhs, hipStream_t s) {
  long long b = (n + RB - 1) / RB;
  const int nb = (int)(b > 2048 ? 2048 : b);
  hipLaunchKernelGGL(k_scale_b, dim3(nb, nrhs), dim3(RB), 0, s, out, in, f, n);
  return hipGetLastError();
}

// f[r] = 1 / sqrt(hn[r]) where hn[r] > tiny2, else 0 (the next basis vector's factor)
__global__ void k_inv_norm_b(const double* __restrict__ hn, double* __restrict__ f, int nrhs, double tiny2) {
  const int r = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (r >= nrhs) return;
  const double h = hn[r];
  f[r] = h > tiny2 ? 1.0 / sqrt(h) : 0.0;
}

hipError_t launch_inv_norm_b(const double* hn, double* f, int nrhs, double tiny2, hipStream_t s) {
  hipLaunchKernelGGL(k_inv_norm_b, dim3((nrhs + 63) / 64), dim3(64), 0, s, hn, f, nrhs, tiny2);
  return hipGetLastError();
}

// STREAM-style copy with 16-byte accesses, one element per thread: the
// attainable-bandwidth probe and the calibration kernel for the traffic counters
template <bool NT>
__global__ void __launch_bounds__(RB) k_stream_copy(u4_t* __restrict__ dst, const u4_t* __restrict__ src,
                                                    long long n16) {
  const long long e = (long long)blockIdx.x * RB + threadIdx.x;
  if (e >= n16) return;
  if constexpr (NT)
    __builtin_nontemporal_store(__builtin_nontemporal_load(src + e), dst + e);
  else
    dst[e] = src[e];
}

hipError_t launch_stream_copy(void* dst, const void* src, long long bytes, bool nontemporal, hipStream_t s) {
  const long long n16 = bytes / 16;
  const long long blocks = (n16 + RB - 1) / RB;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  if (nontemporal)
    hipLaunchKernelGGL(k_stream_copy<true>, dim3((unsigned)blocks), dim3(RB), 0, s, (u4_t*)dst, (const u4_t*)src, n16);
  else
    hipLaunchKernelGGL(k_stream_copy<false>, dim3((unsigned)blocks), dim3(RB), 0, s, (u4_t*)dst, (const u4_t*)src,
                       n16);
  return hipGetLastError();
}

}  // namespace ddq

// Vector kernels shared by the PCG and Lanczos drivers.
#include "reduce.h"

namespace higp {
namespace {

template <typename TA, typename TB>
__global__ __launch_bounds__(kRedThreads) void coldot_kernel(int64_t n, int k, int64_t chunk,
                                                             const TA* __restrict__ A,
                                                             const TB* __restrict__ B,
                                                             double* out, double* work,
                                                             unsigned* counter) {
  __shared__ double sh[kRedThreads];
  const ColLanes L = col_lanes(k);
  const int c = L.c;
  const int r0 = L.r0;
  const int64_t beg = (int64_t)blockIdx.x * chunk;
  const int64_t end = beg + chunk < n ? beg + chunk : n;
  double s = 0.0;
  if (c < k) {
    // Eight rows' loads in flight (two vectors, no stores: 28 µs at n = 1e5,
    // k = 33, against 31 µs with four), products added in row order.
    constexpr int RB = 2 * kRowBatch;
    int64_t i = beg + r0;
    for (; i + (RB - 1) * L.step < end; i += RB * L.step) {
      double a[RB], b[RB];
#pragma unroll
      for (int u = 0; u < RB; ++u) {
        a[u] = ld(A, (i + u * L.step) * k + c);
        b[u] = ld(B, (i + u * L.step) * k + c);
      }
#pragma unroll
      for (int u = 0; u < RB; ++u) s += a[u] * b[u];
    }
    for (; i < end; i += L.step) s += ld(A, i * k + c) * ld(B, i * k + c);
  }
  (void)block_colsum_finish(s, k, work, counter, sh, [&](int col, double tot) { out[col] = tot; });
}

template <typename TX, typename TY>
__global__ void cast_scale_kernel(int64_t count, const TX* __restrict__ x, TY* __restrict__ y,
                                  double a) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x)
    y[e] = (TY)(a * (double)x[e]);
}

}  // namespace

size_t dot_work_doubles(int64_t n, int k) {
  (void)k;
  return (size_t)red_grid(n).blocks * 64;
}

int launch_coldot(int64_t n, int k, const void* A, int ta, const void* B, int tb, double* out,
                  double* work, unsigned* counter, hipStream_t st) {
  const RedGrid g = red_grid(n);
  dim3 grid(g.blocks), block(kRedThreads);
  if (ta == 0 && tb == 0)
    hipLaunchKernelGGL((coldot_kernel<double, double>), grid, block, 0, st, n, k, g.chunk,
                       (const double*)A, (const double*)B, out, work, counter);
  else if (ta == 1 && tb == 1)
    hipLaunchKernelGGL((coldot_kernel<float, float>), grid, block, 0, st, n, k, g.chunk,
                       (const float*)A, (const float*)B, out, work, counter);
  else if (ta == 0 && tb == 1)
    hipLaunchKernelGGL((coldot_kernel<double, float>), grid, block, 0, st, n, k, g.chunk,
                       (const double*)A, (const float*)B, out, work, counter);
  else
    hipLaunchKernelGGL((coldot_kernel<float, double>), grid, block, 0, st, n, k, g.chunk,
                       (const float*)A, (const double*)B, out, work, counter);
  HIGP_HIP_TRY(hipGetLastError());
  return HIGP_OK;
}

int launch_cast_scale(int64_t count, const void* x, int tx, void* y, int ty, double a,
                      hipStream_t st) {
  const int64_t blocks64 = (count + 255) / 256;
  const unsigned blocks = (unsigned)(blocks64 < 2048 ? (blocks64 > 0 ? blocks64 : 1) : 2048);
  if (tx == 0 && ty == 0)
    hipLaunchKernelGGL((cast_scale_kernel<double, double>), dim3(blocks), dim3(256), 0, st, count,
                       (const double*)x, (double*)y, a);
  else if (tx == 0 && ty == 1)
    hipLaunchKernelGGL((cast_scale_kernel<double, float>), dim3(blocks), dim3(256), 0, st, count,
                       (const double*)x, (float*)y, a);
  else if (tx == 1 && ty == 0)
    hipLaunchKernelGGL((cast_scale_kernel<float, double>), dim3(blocks), dim3(256), 0, st, count,
                       (const float*)x, (double*)y, a);
  else
    hipLaunchKernelGGL((cast_scale_kernel<float, float>), dim3(blocks), dim3(256), 0, st, count,
                       (const float*)x, (float*)y, a);
  HIGP_HIP_TRY(hipGetLastError());
  return HIGP_OK;
}

}  // namespace higp

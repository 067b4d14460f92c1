#pragma once
// Area downsampling of the deep guided filtering network (Sec. IV, Fig. 3):
// the high-res input I_h is downsampled to the low-res I_l that the
// low-res network and the guided filtering layer take.  Each low-res pixel
// (i, j) is the mean of its covering high-res rectangle, rows
// floor(i H / h) .. ceil((i + 1) H / h) - 1 and columns likewise (the s x s
// block mean for an integer factor; the rectangles of neighbouring pixels
// overlap by one row or column when the ratio is not an integer).
//
// One workgroup per (plane, low-res row, chunk of low-res columns): the
// threads first sum the covering rows of every high-res column of the
// chunk (coalesced row reads, FP32) into LDS, then each low-res pixel of the
// chunk sums its columns from LDS and divides by its pixel count; the
// result is rounded once to the I/O type.  HBM-bound: every high-res pixel
// is read once (columns shared by two chunks twice).

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gf_internal.h"

namespace gf {
namespace {

constexpr int kDownThreads = 256;
constexpr int kDownCols = 4;  // high-res columns per thread per pass (independent loads)

template <typename T>
__global__ __launch_bounds__(kDownThreads) void downsample_kernel(DownArgs a) {
  extern __shared__ float colsum[];
  const int chunk = blockIdx.x, i = blockIdx.y, plane = blockIdx.z;
  const int H = a.H, W = a.W, h = a.h, w = a.w;
  const int j0 = chunk * a.jc, j1 = min(w, j0 + a.jc);
  const int c_lo = (int)((long long)j0 * W / w);
  const int c_hi = (int)(((long long)j1 * W + w - 1) / w);
  const int r0 = (int)((long long)i * H / h);
  const int r1 = (int)(((long long)(i + 1) * H + h - 1) / h);
  const T* X = reinterpret_cast<const T*>(a.x) + (size_t)plane * H * W;
  for (int base = c_lo + threadIdx.x; base < c_hi; base += kDownThreads * kDownCols) {
    float s[kDownCols];
#pragma unroll
    for (int k = 0; k < kDownCols; ++k) s[k] = 0.f;
    for (int y = r0; y < r1; ++y) {
      const T* row = X + (size_t)y * W;
#pragma unroll
      for (int k = 0; k < kDownCols; ++k) {
        const int x = base + k * kDownThreads;
        if (x < c_hi) s[k] += to_f(row[x]);
      }
    }
#pragma unroll
    for (int k = 0; k < kDownCols; ++k) {
      const int x = base + k * kDownThreads;
      if (x < c_hi) colsum[x - c_lo] = s[k];
    }
  }
  __syncthreads();
  const int j = j0 + (int)threadIdx.x;
  if (j >= j1) return;
  const int x0 = (int)((long long)j * W / w);
  const int x1 = (int)(((long long)(j + 1) * W + w - 1) / w);
  float s = 0.f;
  for (int x = x0; x < x1; ++x) s += colsum[x - c_lo];
  const float cnt = (float)((long long)(r1 - r0) * (x1 - x0));
  T* Y = reinterpret_cast<T*>(a.y) + (size_t)plane * h * w + (size_t)i * w;
  Y[j] = from_f<T>(s / cnt);
}

}  // namespace

template <typename T>
hipError_t downsample_t(const DownArgs& a, hipStream_t s) {
  const dim3 grid((unsigned)((a.w + a.jc - 1) / a.jc), (unsigned)a.h, (unsigned)a.planes);
  prof_begin("gf_downsample", s);
  hipLaunchKernelGGL((downsample_kernel<T>), grid, dim3(kDownThreads),
                     (size_t)a.span * sizeof(float), s, a);
  prof_end(s);
  return hipGetLastError();
}

}  // namespace gf

// Shared definitions of the MI355X (gfx950) ChFSI library.
//
// Storage convention everywhere: complex numbers are interleaved (re, im)
// doubles (double2, 16 bytes), matrices are column-major with an explicit
// leading dimension, exactly like the C-ABI's caller buffers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <stdexcept>
#include <string>

namespace chfsi {

typedef double2 zc;  // complex FP64: x = re, y = im
typedef float2 cc;   // complex FP32

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

// Status codes shared with the C-ABI (see include/chfsi.h).
enum : int {
  ST_OK = 0,
  ST_EINVAL = -1,
  ST_ENOTPD = -2,
  ST_ENOCONV = -3,
  ST_ENAN = -4,
  ST_ENOMEM = -5,
  ST_EHIP = -6,
};

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define CHFSI_HIP(x)                                                                                   \
  do {                                                                                                 \
    hipError_t e_ = (x);                                                                               \
    if (e_ != hipSuccess)                                                                              \
      throw ::chfsi::Error(::chfsi::ST_EHIP, std::string(#x) + ": " + hipGetErrorString(e_) + " (" +  \
                                                 __FILE__ + ":" + std::to_string(__LINE__) + ")");     \
  } while (0)

#define CHFSI_CHECK_LAUNCH() CHFSI_HIP(hipGetLastError())

__host__ __device__ inline zc zmk(double r, double i) { return make_double2(r, i); }
__host__ __device__ inline zc zadd(zc a, zc b) { return make_double2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline zc zsub(zc a, zc b) { return make_double2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline zc zmul(zc a, zc b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
// conj(a) * b
__host__ __device__ inline zc zcmul(zc a, zc b) { return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x); }
__host__ __device__ inline zc zscale(double s, zc a) { return make_double2(s * a.x, s * a.y); }
__host__ __device__ inline zc zconj(zc a) { return make_double2(a.x, -a.y); }
__host__ __device__ inline double zabs2(zc a) { return a.x * a.x + a.y * a.y; }

// Wavefront (64 lanes) sum of a double via cross-lane shuffles.
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block-wide sum for blockDim.x a multiple of 64 (<= 1024); every thread
// gets the result.  `red` must hold blockDim.x/64 doubles.
__device__ inline double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < nw; i++) s += red[i];
  return s;
}

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace chfsi

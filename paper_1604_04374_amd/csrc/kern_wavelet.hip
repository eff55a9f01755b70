// Periodic orthonormal discrete wavelet transforms for Meyer's operator
// representation (section 4.5): the TVIR is expanded in a tensor wavelet
// basis and the expansion is regrouped into windows psi_mu and responses
// c~_mu = sum_lambda c_{lambda,mu} psi_lambda, which are syntheses (inverse
// transforms) of coefficient vectors.
//
// One analysis level on a vector a of length len (periodic):
//   lo[i] = sum_k h[k] a[(2i + k) mod len],  hi[i] = sum_k g[k] a[(2i + k) mod len],
// g[k] = (-1)^k h[L - 1 - k]; coefficients in pyramid order
// [a_J, d_J, ..., d_1].  Synthesis is the transpose, evaluated as a gather:
//   a[p] = sum over k with k = p (mod 2) of h[k] lo[i] + g[k] hi[i],
//   i = ((p - k) / 2) mod (len / 2).
// Vector b's element i lives at base + b * dist + i * stride, so a 2D
// transform is a pass over rows (stride 1) and one over columns (dist 1).
#include <mutex>

#include "pc_internal.hpp"

namespace pc {

// thread -> (vector, element): the faster-moving one is the one adjacent in
// memory, so that consecutive threads touch consecutive addresses
__device__ __forceinline__ void split_index(int64_t t, int64_t count, int64_t len, bool vec_fast, int64_t& b,
                                            int64_t& i) {
  if (vec_fast) {
    b = t % count;
    i = t / count;
  } else {
    i = t % len;
    b = t / len;
  }
}

// one analysis level: src (len elements per vector, strided) -> lo into dst
// (len/2, contiguous per vector, distance len/2) and hi into out at
// positions [len/2, len) (strided)
__global__ __launch_bounds__(256) void k_dwt_level(const float* __restrict__ src, int64_t s_stride, int64_t s_dist,
                                                   float* __restrict__ lo_dst, int64_t l_dist,
                                                   float* __restrict__ out, int64_t o_stride, int64_t o_dist,
                                                   int64_t count, int64_t len, WaveletFilter f, int vec_fast) {
  const int64_t half = len / 2;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count * half) return;
  int64_t b, i;
  split_index(t, count, half, vec_fast != 0, b, i);
  const float* a = src + b * s_dist;
  float lo = 0.f, hi = 0.f;
  for (int k = 0; k < f.taps; ++k) {
    int64_t p = 2 * i + k;
    p = p % len;
    const float v = a[p * s_stride];
    lo = fmaf(f.h[k], v, lo);
    hi = fmaf(f.g[k], v, hi);
  }
  lo_dst[b * l_dist + i] = lo;
  out[b * o_dist + (half + i) * o_stride] = hi;
}

// one synthesis level: lo (contiguous, distance l_dist) and hi (strided in c,
// positions [half, 2 half)) -> dst (2 half elements, strided)
__global__ __launch_bounds__(256) void k_idwt_level(const float* __restrict__ lo_src, int64_t l_stride, int64_t l_dist,
                                                    const float* __restrict__ c, int64_t c_stride, int64_t c_dist,
                                                    float* __restrict__ dst, int64_t d_stride, int64_t d_dist,
                                                    int64_t count, int64_t half, WaveletFilter f, int vec_fast) {
  const int64_t len = 2 * half;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count * len) return;
  int64_t b, p;
  split_index(t, count, len, vec_fast != 0, b, p);
  const float* lo = lo_src + b * l_dist;
  const float* hi = c + b * c_dist + half * c_stride;
  float acc = 0.f;
  for (int k = (int)(p & 1); k < f.taps; k += 2) {
    int64_t i = (p - k) / 2;  // p - k is even
    i %= half;
    if (i < 0) i += half;
    acc = fmaf(f.h[k], lo[i * l_stride], acc);
    acc = fmaf(f.g[k], hi[i * c_stride], acc);
  }
  dst[b * d_dist + p * d_stride] = acc;
}

// out[b][i] = in[b][i] for i < len (strided on both sides)
__global__ __launch_bounds__(256) void k_copy_strided(const float* __restrict__ in, int64_t i_stride, int64_t i_dist,
                                                      float* __restrict__ out, int64_t o_stride, int64_t o_dist,
                                                      int64_t count, int64_t len, int vec_fast) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count * len) return;
  int64_t b, i;
  split_index(t, count, len, vec_fast != 0, b, i);
  out[b * o_dist + i * o_stride] = in[b * i_dist + i * i_stride];
}

static inline unsigned blocks_n(int64_t n) { return (unsigned)((n + 255) / 256); }

LaunchStatus launch_wavelet(bool synthesis, int64_t n, int levels, const WaveletFilter& f, int64_t count,
                            int64_t stride, int64_t dist, const float* in, float* out, float* s1, float* s2,
                            hipStream_t s) {
  const int vf = dist < stride ? 1 : 0;
  hipError_t e = hipSuccess;
  if (!synthesis) {
    // level j reads A_j (in, then s1 / s2 alternately, contiguous with
    // distance len) and writes lo to the other scratch buffer, hi to out
    const float* src = in;
    int64_t ss = stride, sd = dist;
    int64_t len = n;
    for (int j = 0; j < levels && e == hipSuccess; ++j) {
      float* lo = (j % 2 == 0) ? s1 : s2;
      hipLaunchKernelGGL(k_dwt_level, dim3(blocks_n(count * (len / 2))), dim3(256), 0, s, src, ss, sd, lo, len / 2,
                         out, stride, dist, count, len, f, j == 0 ? vf : 0);
      e = hipGetLastError();
      src = lo;
      ss = 1;
      sd = len / 2;
      len /= 2;
    }
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_copy_strided, dim3(blocks_n(count * len)), dim3(256), 0, s, src, ss, sd, out, stride,
                         dist, count, len, vf);
      e = hipGetLastError();
    }
    return e;
  }
  // synthesis: the approximation starts in `in` (first n >> levels entries)
  // and alternates between s1 and s2; the last level writes out
  const float* lo = in;
  int64_t ls = stride, ld = dist;
  int64_t half = n >> levels;
  for (int j = 0; j < levels && e == hipSuccess; ++j) {
    const bool last = j == levels - 1;
    float* dst = last ? out : ((j % 2 == 0) ? s1 : s2);
    const int64_t ds = last ? stride : 1, dd = last ? dist : 2 * half;
    hipLaunchKernelGGL(k_idwt_level, dim3(blocks_n(count * 2 * half)), dim3(256), 0, s, lo, ls, ld, in, stride, dist,
                       dst, ds, dd, count, half, f, last ? vf : 0);
    e = hipGetLastError();
    lo = dst;
    ls = 1;
    ld = 2 * half;
    half *= 2;
  }
  if (levels == 0 && e == hipSuccess) {
    hipLaunchKernelGGL(k_copy_strided, dim3(blocks_n(count * n)), dim3(256), 0, s, in, stride, dist, out, stride,
                       dist, count, n, vf);
    e = hipGetLastError();
  }
  return e;
}

// ---------------------------------------------------------------------------
// Allocation-free transforms: the two ping-pong buffers live in a fixed
// device array instead of the library's grow-only scratch.  Each device
// holds its own copy of the array; its address is looked up once per device
// (with that device current) and kept.  The array is shared by every such
// call on a device, so calls that overlap on one device race; every entry a
// level reads was written by the level before it in the same call, so
// nothing needs clearing between calls.
// ---------------------------------------------------------------------------
static __device__ __align__(256) float scratch[WAVELET_STATIC_FLOATS];

namespace {
std::mutex g_static_mu;
float* g_static_ptr[64] = {};  // per device
}  // namespace

LaunchStatus launch_wavelet_static(bool synthesis, int64_t n, int levels, const WaveletFilter& f, int64_t count,
                                   int64_t stride, int64_t dist, const float* in, float* out, hipStream_t s) {
  if (count * (n / 2) > WAVELET_STATIC_FLOATS / 2) return hipErrorInvalidValue;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  float* base = nullptr;
  {
    std::lock_guard<std::mutex> g(g_static_mu);
    if (!g_static_ptr[dev]) {
      void* ptr = nullptr;
      e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess) return e;
      g_static_ptr[dev] = static_cast<float*>(ptr);
    }
    base = g_static_ptr[dev];
  }
  float* s1 = base;
  float* s2 = base + WAVELET_STATIC_FLOATS / 2;
  return launch_wavelet(synthesis, n, levels, f, count, stride, dist, in, out, s1, s2, s);
}

}  // namespace pc

// Construction of the impulse responses h_k from a TVIR (section 4): the L2
// projection of every TVIR row onto the span of the windows (section 4.2,
// the B-spline case of Corollary 4.3) and the interpolation at m nodes
// (section 4.4).  For a lag row T(x, .):
//   projection:     (W W^T) c(x) = W T(x, .)^T
//   interpolation:  E c(x) = (T(x, y_i))_i,   E[i][k] = w_k(y_i)
// and h_k[x] = c_k(x) / n.
//
// The contraction W T^T (rows x n times n x m) is the one dense product of
// the path: it runs on the matrix cores in FP32 (v_mfma_f32_16x16x4f32), split
// along n into chunks whose partial sums are added in float64; the m x m
// factorisations and the per-row solves are float64.
#include "pc_internal.hpp"

namespace pc {

typedef float floatx4 __attribute__((ext_vector_type(4)));

// part[split][r][c] = sum over the split's chunk of j of A[r][j] B[c][j].
// A: rows x K, B: cols x K, both row-major with K contiguous, K % 16 == 0,
// 16-byte aligned rows.  Workgroup: 4 waves x GEMM_WAVE_ROWS rows, 32
// columns; a wave holds GEMM_WAVE_ROWS / 16 row blocks x 2 column blocks of
// 16 x 16 outputs, so each 16-byte load of B serves that many row blocks
// (B, the windows, is re-read by every workgroup; A, the TVIR band, is
// streamed once).  Each lane loads 4 consecutive k of its rows (and of its
// two columns) and feeds them to 4 consecutive MFMA steps, so one 16-k step
// of the loop covers k0 + 4g + s for lane group g < 4 and step s < 4 on both
// operands alike.
__global__ __launch_bounds__(256) void k_gemm_nt_f32(const float* __restrict__ A, int64_t rows,
                                                     const float* __restrict__ B, int cols, int64_t K,
                                                     float* __restrict__ part) {
  constexpr int RT = GEMM_WAVE_ROWS / 16;  // row blocks per wave
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, li = lane & 15;
  const int64_t r0 = (int64_t)blockIdx.x * GEMM_ROWS + (int64_t)wave * GEMM_WAVE_ROWS;
  const int ca = blockIdx.y * GEMM_COLS + li, cb = ca + 16;
  const bool aok = ca < cols, bok = cb < cols;
  const int64_t k_begin = (int64_t)blockIdx.z * GEMM_CHUNK;
  const int64_t k_end = k_begin + GEMM_CHUNK < K ? k_begin + GEMM_CHUNK : K;
  // out-of-range rows and columns read row 0 (valid memory) and are zeroed
  // by a factor, so that every load is one unconditional 16-byte access
  const float4* Ar[RT];
  float fa[RT];
#pragma unroll
  for (int b = 0; b < RT; ++b) {
    const int64_t r = r0 + 16 * b + li;
    const bool rok = r < rows;
    Ar[b] = reinterpret_cast<const float4*>(A + (rok ? r : 0) * K);
    fa[b] = rok ? 1.f : 0.f;
  }
  const float4* Ba = reinterpret_cast<const float4*>(B + (int64_t)(aok ? ca : 0) * K);
  const float4* Bb = reinterpret_cast<const float4*>(B + (int64_t)(bok ? cb : 0) * K);
  const float fx = aok ? 1.f : 0.f, fy = bok ? 1.f : 0.f;
  auto scale = [](float4 v, float f) { return make_float4(v.x * f, v.y * f, v.z * f, v.w * f); };
  floatx4 acc0[RT], acc1[RT];
#pragma unroll
  for (int b = 0; b < RT; ++b) {
    acc0[b] = floatx4{0.f, 0.f, 0.f, 0.f};
    acc1[b] = floatx4{0.f, 0.f, 0.f, 0.f};
  }
  // operands of step k0 + 16 load while the MFMAs of step k0 issue
  int64_t q = (k_begin >> 2) + g;  // float4 index of k0 + 4g
  float4 an[RT];
#pragma unroll
  for (int b = 0; b < RT; ++b) an[b] = Ar[b][q];
  float4 xn = Ba[q], yn = Bb[q];
  for (int64_t k0 = k_begin; k0 < k_end; k0 += 16) {
    float4 a[RT];
#pragma unroll
    for (int b = 0; b < RT; ++b) a[b] = scale(an[b], fa[b]);
    const float4 x = scale(xn, fx), y = scale(yn, fy);
    q += 4;
    if (k0 + 16 < k_end) {
#pragma unroll
      for (int b = 0; b < RT; ++b) an[b] = Ar[b][q];
      xn = Ba[q];
      yn = Bb[q];
    }
#pragma unroll
    for (int b = 0; b < RT; ++b) {
      acc0[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[b].x, x.x, acc0[b], 0, 0, 0);
      acc1[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[b].x, y.x, acc1[b], 0, 0, 0);
      acc0[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[b].y, x.y, acc0[b], 0, 0, 0);
      acc1[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[b].y, y.y, acc1[b], 0, 0, 0);
      acc0[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[b].z, x.z, acc0[b], 0, 0, 0);
      acc1[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[b].z, y.z, acc1[b], 0, 0, 0);
      acc0[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[b].w, x.w, acc0[b], 0, 0, 0);
      acc1[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[b].w, y.w, acc1[b], 0, 0, 0);
    }
  }
  // output block element (i, j) sits in lane j + 16 (i / 4), item i % 4
  float* P = part + (int64_t)blockIdx.z * rows * cols;
#pragma unroll
  for (int b = 0; b < RT; ++b)
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const int64_t row = r0 + 16 * b + 4 * g + it;
      if (row < rows) {
        if (aok) P[row * cols + ca] = acc0[b][it];
        if (bok) P[row * cols + cb] = acc1[b][it];
      }
    }
}

// out[i] = sum_s part[s][i] in float64
__global__ __launch_bounds__(256) void k_sum_splits(const float* __restrict__ part, int splits, int64_t n,
                                                    double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int t = 0; t < splits; ++t) s += (double)part[(int64_t)t * n + i];
  out[i] = s;
}

// In-place Cholesky G = L L^T (lower triangle, m <= CONSTRUCT_MAX_M), one
// workgroup; *fail = 1 if a pivot is not above 1e-12 of its diagonal entry
// (the windows are numerically dependent).
__global__ __launch_bounds__(256) void k_cholesky(double* __restrict__ G, int m, int* __restrict__ fail) {
  __shared__ double S[CONSTRUCT_MAX_M * CONSTRUCT_MAX_M];
  __shared__ int bad;
  for (int i = threadIdx.x; i < m * m; i += blockDim.x) S[i] = G[i];
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  for (int j = 0; j < m; ++j) {
    if (threadIdx.x == 0) {
      const double g = S[j * m + j];
      double d = g;
      for (int p = 0; p < j; ++p) d -= S[j * m + p] * S[j * m + p];
      if (!(d > 1e-12 * g)) {
        bad = 1;
        d = 1.0;
      }
      S[j * m + j] = sqrt(d);
    }
    __syncthreads();
    for (int i = j + 1 + threadIdx.x; i < m; i += blockDim.x) {
      double v = S[i * m + j];
      for (int p = 0; p < j; ++p) v -= S[i * m + p] * S[j * m + p];
      S[i * m + j] = v / S[j * m + j];
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < m * m; i += blockDim.x) G[i] = S[i];
  if (threadIdx.x == 0) *fail = bad;
}

// In-place LU with partial pivoting of E (m x m): L unit lower, U upper,
// perm[i] = original row of pivot row i; *fail = 1 when a pivot is not above
// 1e-12 of the largest entry of E.
__global__ __launch_bounds__(256) void k_lu(double* __restrict__ E, int m, int* __restrict__ perm,
                                            int* __restrict__ fail) {
  __shared__ double S[CONSTRUCT_MAX_M * CONSTRUCT_MAX_M];
  __shared__ int pr[CONSTRUCT_MAX_M];
  __shared__ int bad, piv;
  __shared__ double emax;
  for (int i = threadIdx.x; i < m * m; i += blockDim.x) S[i] = E[i];
  for (int i = threadIdx.x; i < m; i += blockDim.x) pr[i] = i;
  __syncthreads();
  if (threadIdx.x == 0) {
    bad = 0;
    double a = 0.0;
    for (int i = 0; i < m * m; ++i) a = fmax(a, fabs(S[i]));
    emax = a;
  }
  __syncthreads();
  for (int j = 0; j < m; ++j) {
    if (threadIdx.x == 0) {
      int best = j;
      for (int i = j + 1; i < m; ++i)
        if (fabs(S[i * m + j]) > fabs(S[best * m + j])) best = i;
      if (!(fabs(S[best * m + j]) > 1e-12 * emax)) bad = 1;
      piv = best;
    }
    __syncthreads();
    if (piv != j) {
      for (int c = threadIdx.x; c < m; c += blockDim.x) {
        const double t = S[j * m + c];
        S[j * m + c] = S[piv * m + c];
        S[piv * m + c] = t;
      }
      if (threadIdx.x == 0) {
        const int t = pr[j];
        pr[j] = pr[piv];
        pr[piv] = t;
      }
    }
    __syncthreads();
    const double d = S[j * m + j];
    if (d != 0.0) {
      for (int i = j + 1 + threadIdx.x; i < m; i += blockDim.x) S[i * m + j] /= d;
      __syncthreads();
      for (int e = threadIdx.x; e < (m - j - 1) * (m - j - 1); e += blockDim.x) {
        const int i = j + 1 + e / (m - j - 1), c = j + 1 + e % (m - j - 1);
        S[i * m + c] -= S[i * m + j] * S[j * m + c];
      }
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < m * m; i += blockDim.x) E[i] = S[i];
  for (int i = threadIdx.x; i < m; i += blockDim.x) perm[i] = pr[i];
  if (threadIdx.x == 0) *fail = bad;
}

// One thread per TVIR row r: solve for c(x_r) in float64 in the row's slot of
// `work` (m values), starting from the row of `src`, and write
// h[k][lags[r]] = c_k / n.
//   LU = false: F is the Cholesky factor L of the Gram matrix (L, then L^T).
//   LU = true:  F holds unit-lower L and U with the row permutation perm.
template <bool LU>
__global__ __launch_bounds__(256) void k_row_solve(const double* __restrict__ F, const int* __restrict__ perm, int m,
                                                   const double* __restrict__ src, double* __restrict__ work,
                                                   int64_t rows, const int64_t* __restrict__ lags, int64_t n,
                                                   float* __restrict__ h) {
  __shared__ double S[CONSTRUCT_MAX_M * CONSTRUCT_MAX_M];
  for (int i = threadIdx.x; i < m * m; i += blockDim.x) S[i] = F[i];
  __syncthreads();
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  const double* a = src + r * m;
  double* b = work + r * m;
  if (LU) {
    for (int i = 0; i < m; ++i) b[i] = a[perm[i]];
    for (int i = 0; i < m; ++i) {  // L y = P t, L unit lower
      double v = b[i];
      for (int p = 0; p < i; ++p) v -= S[i * m + p] * b[p];
      b[i] = v;
    }
    for (int i = m - 1; i >= 0; --i) {  // U c = y
      double v = b[i];
      for (int p = i + 1; p < m; ++p) v -= S[i * m + p] * b[p];
      b[i] = v / S[i * m + i];
    }
  } else {
    for (int i = 0; i < m; ++i) {  // L y = b
      double v = a[i];
      for (int p = 0; p < i; ++p) v -= S[i * m + p] * b[p];
      b[i] = v / S[i * m + i];
    }
    for (int i = m - 1; i >= 0; --i) {  // L^T c = y
      double v = b[i];
      for (int p = i + 1; p < m; ++p) v -= S[p * m + i] * b[p];
      b[i] = v / S[i * m + i];
    }
  }
  const int64_t l = lags[r];
  const double inv_n = 1.0 / (double)n;
  for (int k = 0; k < m; ++k) h[(int64_t)k * n + l] = (float)(b[k] * inv_n);
}

__global__ __launch_bounds__(256) void k_fill_zero(float* __restrict__ x, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0.f;
}

// E[i][k] = W[k][nodes[i]] (float64), and the samples as float64 rows
__global__ __launch_bounds__(256) void k_node_matrix(const float* __restrict__ W, int m, int64_t n,
                                                     const int64_t* __restrict__ nodes, double* __restrict__ E) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * m) return;
  const int i = e / m, k = e % m;
  E[e] = (double)W[(int64_t)k * n + nodes[i]];
}

__global__ __launch_bounds__(256) void k_to_double(const float* __restrict__ x, int64_t n, double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (double)x[i];
}

// out[k][l] = in[k][-l] on every axis (lag layout), 1D (n1 == 1) or 2D
__global__ __launch_bounds__(256) void k_flip(const float* __restrict__ in, float* __restrict__ out, int64_t count,
                                              int64_t n0, int64_t n1) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= count * n0 * n1) return;
  const int64_t k = g / (n0 * n1), rem = g % (n0 * n1);
  const int64_t i = rem / n1, j = rem % n1;
  out[g] = in[(k * n0 + (n0 - i) % n0) * n1 + (n1 - j) % n1];
}

static inline unsigned blocks_of(int64_t n) { return (unsigned)((n + 255) / 256); }

LaunchStatus launch_gemm_nt(const float* A, int64_t rows, const float* B, int cols, int64_t K, float* part,
                            hipStream_t s) {
  const dim3 grid((unsigned)((rows + GEMM_ROWS - 1) / GEMM_ROWS), (unsigned)((cols + GEMM_COLS - 1) / GEMM_COLS),
                  (unsigned)gemm_splits(K));
  hipLaunchKernelGGL(k_gemm_nt_f32, grid, dim3(256), 0, s, A, rows, B, cols, K, part);
  return hipGetLastError();
}

LaunchStatus launch_sum_splits(const float* part, int splits, int64_t n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_splits, dim3(blocks_of(n)), dim3(256), 0, s, part, splits, n, out);
  return hipGetLastError();
}

LaunchStatus launch_cholesky(double* G, int m, int* fail, hipStream_t s) {
  hipLaunchKernelGGL(k_cholesky, dim3(1), dim3(256), 0, s, G, m, fail);
  return hipGetLastError();
}

LaunchStatus launch_lu(double* E, int m, int* perm, int* fail, hipStream_t s) {
  hipLaunchKernelGGL(k_lu, dim3(1), dim3(256), 0, s, E, m, perm, fail);
  return hipGetLastError();
}

LaunchStatus launch_row_solve(bool lu, const double* F, const int* perm, int m, const double* src, double* work,
                              int64_t rows, const int64_t* lags, int64_t n, float* h, hipStream_t s) {
  if (lu)
    hipLaunchKernelGGL(k_row_solve<true>, dim3(blocks_of(rows)), dim3(256), 0, s, F, perm, m, src, work, rows, lags,
                       n, h);
  else
    hipLaunchKernelGGL(k_row_solve<false>, dim3(blocks_of(rows)), dim3(256), 0, s, F, perm, m, src, work, rows,
                       lags, n, h);
  return hipGetLastError();
}

LaunchStatus launch_fill_zero(float* x, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_zero, dim3(blocks_of(n)), dim3(256), 0, s, x, n);
  return hipGetLastError();
}

LaunchStatus launch_node_matrix(const float* W, int m, int64_t n, const int64_t* nodes, double* E, hipStream_t s) {
  hipLaunchKernelGGL(k_node_matrix, dim3(blocks_of((int64_t)m * m)), dim3(256), 0, s, W, m, n, nodes, E);
  return hipGetLastError();
}

LaunchStatus launch_to_double(const float* x, int64_t n, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_to_double, dim3(blocks_of(n)), dim3(256), 0, s, x, n, y);
  return hipGetLastError();
}

LaunchStatus launch_flip(const float* in, float* out, int64_t count, int64_t n0, int64_t n1, hipStream_t s) {
  hipLaunchKernelGGL(k_flip, dim3(blocks_of(count * n0 * n1)), dim3(256), 0, s, in, out, count, n0, n1);
  return hipGetLastError();
}

}  // namespace pc

// Overlap-add kernel of the sectioned 2D evaluation (the
// compact-support complexity lemma of section 3.5, Lemma 3.2).
//
// A term whose window has the box [o, o + p) (per axis, on the torus) and
// whose impulse response has the lag box [a, a + q) is evaluated on a
// section of M >= p + q - 1 samples per axis: the windowed input of the box
// convolved with the shifted response is a linear convolution there, and
// its nonzero part, of p + q - 1 samples, lands at o + a.  The adjoint reads
// the input at o + a and writes the window box.  The section transforms run
// in the single-term 2D kernels, whose row-forward pass reads each input box
// in place; the overlap-add of the output boxes is here.
#include "pc_internal.hpp"

namespace pc {

// One workgroup per (tile, image) of SEC_TILE_R x SEC_TILE_C pixels, each
// thread SEC_ROWS_PER_THREAD rows of one column: every pixel is the sum, in
// section order, of the sections whose output box covers it.  The sections
// of a tile's list are taken SEC_GROUP at a time, every sample of the group
// loaded before any is added (one wait per group instead of one per
// section), then added in list order.
//
// Tiles are numbered XCD-major: workgroups are dispatched round-robin over
// the 8 XCDs, so workgroup x runs on XCD x mod 8, and that XCD is given a
// run of consecutive tiles (row-major: mostly horizontal neighbours).  A
// section's row segment starts at an arbitrary column, so the 128-byte
// lines at a tile's left and right edges are shared with the neighbouring
// tiles; on one XCD they are fetched into its L2 once.
constexpr int SEC_XCDS = 8;
__device__ __forceinline__ int xcd_major_tile(int x, int n) {
  const int q = n / SEC_XCDS;
  return x < q * SEC_XCDS ? (x % SEC_XCDS) * q + x / SEC_XCDS : x;
}
constexpr int SEC_THREADS = 128, SEC_ROWS_PER_THREAD = SEC_TILE_R * SEC_TILE_C / SEC_THREADS,
              SEC_ROW_STEP = SEC_THREADS / SEC_TILE_C, SEC_GROUP = 4;
__global__ __launch_bounds__(SEC_THREADS) void k_sec_scatter(
    const SecTerm* __restrict__ terms, const float* __restrict__ S, float* __restrict__ y_arg,
    float* const* __restrict__ yp, int N1, int N2, int tiles2, const int* __restrict__ toff,
    const int* __restrict__ titems, int adjoint) {
  float* y = yp ? *yp : y_arg;
  const int tile = xcd_major_tile(blockIdx.x, gridDim.x);
  const int64_t b = blockIdx.y;
  const int i10 = (tile / tiles2) * SEC_TILE_R + (int)threadIdx.x / SEC_TILE_C;  // rows i10 + SEC_ROW_STEP r
  const int i2 = (tile % tiles2) * SEC_TILE_C + (int)threadIdx.x % SEC_TILE_C;
  float acc[SEC_ROWS_PER_THREAD];
#pragma unroll
  for (int r = 0; r < SEC_ROWS_PER_THREAD; ++r) acc[r] = 0.f;
  const int j0 = toff[tile], j1 = toff[tile + 1];
  for (int j = j0; j < j1; j += SEC_GROUP) {
    float v[SEC_GROUP][SEC_ROWS_PER_THREAD];
#pragma unroll
    for (int g = 0; g < SEC_GROUP; ++g) {
      // a sample outside the section's box, or past the list's end, is zero
      bool in2 = false;
      const float* Sb = S;  // the section's column d2 of image b
      int64_t M2 = 0;
      int s1 = 0, e1 = 0;
      if (j + g < j1) {
        const SecTerm tm = terms[titems[j + g]];
        const int s2 = adjoint ? tm.sa2 : tm.sf2, e2 = adjoint ? tm.ea2 : tm.ef2;
        s1 = adjoint ? tm.sa1 : tm.sf1;
        e1 = adjoint ? tm.ea1 : tm.ef1;
        int d2 = i2 - s2;
        if (d2 < 0) d2 += N2;
        in2 = d2 < e2;
        M2 = tm.M2;
        Sb = S + tm.off + b * tm.M1 * tm.M2 + d2;
      }
#pragma unroll
      for (int r = 0; r < SEC_ROWS_PER_THREAD; ++r) {
        int d1 = i10 + SEC_ROW_STEP * r - s1;
        if (d1 < 0) d1 += N1;
        v[g][r] = in2 && d1 < e1 ? Sb[(int64_t)d1 * M2] : 0.f;
      }
    }
#pragma unroll
    for (int g = 0; g < SEC_GROUP; ++g)
#pragma unroll
      for (int r = 0; r < SEC_ROWS_PER_THREAD; ++r) acc[r] += v[g][r];
  }
#pragma unroll
  for (int r = 0; r < SEC_ROWS_PER_THREAD; ++r) y[(b * N1 + i10 + SEC_ROW_STEP * r) * N2 + i2] = acc[r];
}

LaunchStatus launch_sec_scatter(const Sec2D& q, float* y, bool adjoint, int64_t batch, hipStream_t s, Tracer* tr,
                                float* const* yp) {
  TraceScope ts(tr, "sec_scatter", s);
  const int tiles = (q.N1 / SEC_TILE_R) * q.tiles2;
  hipLaunchKernelGGL(k_sec_scatter, dim3((unsigned)tiles, (unsigned)batch), dim3(SEC_THREADS), 0, s,
                     q.terms, q.Sout, y, yp, q.N1, q.N2, q.tiles2, adjoint ? q.ta_off : q.tf_off,
                     adjoint ? q.ta_items : q.tf_items, adjoint ? 1 : 0);
  return hipGetLastError();
}

}  // namespace pc

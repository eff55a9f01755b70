// Gather and overlap-add kernels of the sectioned 2D evaluation (the
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

// One thread per output pixel, one workgroup per (tile, image): the sum, in
// section order, of the sections whose output box covers the pixel.
__global__ __launch_bounds__(SEC_TILE_R * SEC_TILE_C) void k_sec_scatter(
    const SecTerm* __restrict__ terms, const float* __restrict__ S, float* __restrict__ y, int N1, int N2,
    int tiles2, const int* __restrict__ toff, const int* __restrict__ titems, int adjoint) {
  const int tile = blockIdx.x;
  const int64_t b = blockIdx.y;
  const int i1 = (tile / tiles2) * SEC_TILE_R + (int)threadIdx.x / SEC_TILE_C;
  const int i2 = (tile % tiles2) * SEC_TILE_C + (int)threadIdx.x % SEC_TILE_C;
  float acc = 0.f;
  for (int j = toff[tile]; j < toff[tile + 1]; ++j) {
    const SecTerm tm = terms[titems[j]];
    const int s1 = adjoint ? tm.sa1 : tm.sf1, s2 = adjoint ? tm.sa2 : tm.sf2;
    const int e1 = adjoint ? tm.ea1 : tm.ef1, e2 = adjoint ? tm.ea2 : tm.ef2;
    int d1 = i1 - s1;
    if (d1 < 0) d1 += N1;
    int d2 = i2 - s2;
    if (d2 < 0) d2 += N2;
    if (d1 < e1 && d2 < e2) acc += S[tm.off + (b * tm.M1 + d1) * tm.M2 + d2];
  }
  y[(b * N1 + i1) * N2 + i2] = acc;
}

LaunchStatus launch_sec_scatter(const Sec2D& q, float* y, bool adjoint, int64_t batch, hipStream_t s, Tracer* tr) {
  TraceScope ts(tr, "sec_scatter", s);
  const int tiles = (q.N1 / SEC_TILE_R) * q.tiles2;
  hipLaunchKernelGGL(k_sec_scatter, dim3((unsigned)tiles, (unsigned)batch), dim3(SEC_TILE_R * SEC_TILE_C), 0, s,
                     q.terms, q.Sout, y, q.N1, q.N2, q.tiles2, adjoint ? q.ta_off : q.tf_off,
                     adjoint ? q.ta_items : q.tf_items, adjoint ? 1 : 0);
  return hipGetLastError();
}

}  // namespace pc

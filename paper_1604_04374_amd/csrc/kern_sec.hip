// Gather and overlap-add kernels of the sectioned 2D evaluation (the
// compact-support complexity lemma of section 3.5, Lemma 3.2).
//
// A term whose window has the box [o, o + p) (per axis, on the torus) and
// whose impulse response has the lag box [a, a + q) is evaluated on a
// section of M >= p + q - 1 samples per axis: the windowed input of the box
// convolved with the shifted response is a linear convolution there, and
// its nonzero part, of p + q - 1 samples, lands at o + a.  The adjoint reads
// the input at o + a and writes the window box.  The section transforms run
// in the single-term 2D kernels; these kernels move the boxes in and out.
#include "pc_internal.hpp"

namespace pc {

// One workgroup per (section, image, row): staging row <- input row of the
// box, both axes wrapped.
__global__ __launch_bounds__(256) void k_sec_gather(const SecTerm* __restrict__ terms, const float* __restrict__ x,
                                                    float* __restrict__ S, int N1, int N2, int64_t batch,
                                                    int adjoint) {
  const SecTerm tm = terms[blockIdx.y];
  const int64_t r = blockIdx.x;  // b * M1 + i
  if (r >= batch * tm.M1) return;
  const int64_t b = r / tm.M1;
  const int i = (int)(r % tm.M1);
  const int g1 = adjoint ? tm.ga1 : tm.gf1;
  const int g2 = adjoint ? tm.ga2 : tm.gf2;
  int i1 = g1 + i;  // g1 < N1 and i < M1 <= N1
  if (i1 >= N1) i1 -= N1;
  const float* src = x + (b * N1 + i1) * N2;
  float* dst = S + tm.off + r * tm.M2;
  for (int j = threadIdx.x; j < tm.M2; j += blockDim.x) {
    int j2 = g2 + j;
    if (j2 >= N2) j2 -= N2;
    dst[j] = src[j2];
  }
}

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

LaunchStatus launch_sec_gather(const Sec2D& q, const float* x, bool adjoint, int64_t batch, hipStream_t s,
                               Tracer* tr) {
  TraceScope ts(tr, "sec_gather", s);
  hipLaunchKernelGGL(k_sec_gather, dim3((unsigned)(batch * q.max_m1), (unsigned)q.n_sec), dim3(256), 0, s, q.terms,
                     x, q.Sin, q.N1, q.N2, batch, adjoint ? 1 : 0);
  return hipGetLastError();
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

// Host-side check library (tests only): exposes the radix butterflies of
// tbs_fft.hpp to the CPU test-suite.  Not part of libtbs.
#include "../tbs_fft.hpp"

namespace {
template <int R, bool INV>
void run(const double* in, double* out) {
  tbs::cx<double> a[R];
  for (int i = 0; i < R; ++i) a[i] = {in[2 * i], in[2 * i + 1]};
  tbs::dft<R, INV>(a);
  for (int i = 0; i < R; ++i) {
    out[2 * i] = a[i].x;
    out[2 * i + 1] = a[i].y;
  }
}
}  // namespace

extern "C" int tbs_hostcheck_dft(int R, int inv, const double* in, double* out) {
#define C(r)                                          \
  case r:                                             \
    if (inv) run<r, true>(in, out); else run<r, false>(in, out); \
    return 0;
  switch (R) {
    C(2) C(3) C(4) C(5) C(8) C(16)
    default: return -1;
  }
#undef C
}

extern "C" int tbs_hostcheck_stages(int M, int E, int* radices) {
  tbs::Stages s = tbs::make_stages(M, E);
  for (int i = 0; i < s.n; ++i) radices[i] = s.r[i];
  return s.n;
}

// Host-side check library (tests only): exposes the radix butterflies, the
// stage plans and the exchange index maps of tbs_fft.hpp to the CPU
// test-suite.  Not part of libtbs.
#include <cmath>
#include <vector>

#include "../tbs_bf16.hpp"
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

namespace {
template <int R, bool INV>
void run_half(const double* in, double* out) {
  tbs::cx<double> a[R];
  for (int i = 0; i < R; ++i) a[i] = i < R / 2 ? tbs::cx<double>{in[2 * i], in[2 * i + 1]} : tbs::cx<double>{0.0, 0.0};
  tbs::dft_half<R, INV>(a);
  for (int i = 0; i < R; ++i) {
    out[2 * i] = a[i].x;
    out[2 * i + 1] = a[i].y;
  }
}
}  // namespace

// The first-stage DFTs of a zero-padded line: in holds the R/2 nonzero
// inputs, out the R outputs.
extern "C" int tbs_hostcheck_dft_half(int R, int inv, const double* in, double* out) {
#define C(r)                                                      \
  case r:                                                         \
    if (inv) run_half<r, true>(in, out); else run_half<r, false>(in, out); \
    return 0;
  switch (R) {
    C(2) C(4) C(8) C(16)
    default: return -1;
  }
#undef C
}

extern "C" int tbs_hostcheck_stages(int M, int E, int* radices) {
  tbs::Stages s = tbs::make_stages(M, E);
  for (int i = 0; i < s.n; ++i) radices[i] = s.r[i];
  return s.n;
}

namespace {
template <int R, bool INV>
void dft_n(tbs::cx<double>* a) {
  tbs::cx<double> b[R];
  for (int i = 0; i < R; ++i) b[i] = a[i];
  tbs::dft<R, INV>(b);
  for (int i = 0; i < R; ++i) a[i] = b[i];
}

template <bool INV>
void dft_rt(int R, tbs::cx<double>* a) {
  switch (R) {
    case 2: dft_n<2, INV>(a); break;
    case 3: dft_n<3, INV>(a); break;
    case 4: dft_n<4, INV>(a); break;
    case 5: dft_n<5, INV>(a); break;
    case 8: dft_n<8, INV>(a); break;
    case 16: dft_n<16, INV>(a); break;
  }
}
}  // namespace

// Runs the device transform's data flow on the host: TPT = M/E emulated
// threads with E registers each in the strided layout, every stage's
// butterflies, and between stages either the exchange through a shared
// array at the slots the device uses for 8-byte elements (xwrite_slot,
// read back at xread_slot) or, for local stages, the register renaming
// local_register.  out receives the transform (natural
// order); *n_exchanges / *n_local count the two kinds of hand-over.
extern "C" int tbs_hostcheck_fft(int M, int E, int inv, const double* in, double* out,
                                 int* n_exchanges, int* n_local) {
  if (M % E) return -1;
  const tbs::Stages st = tbs::make_stages(M, E);
  if (st.n <= 0) return -1;
  const int TPT = M / E;
  std::vector<tbs::cx<double>> v((size_t)M), w((size_t)M), sh((size_t)tbs::lds_len(M, 1, 8));
  for (int t = 0; t < TPT; ++t)
    for (int j = 0; j < E; ++j) v[(size_t)t * E + j] = {in[2 * (t + j * TPT)], in[2 * (t + j * TPT) + 1]};
  int L = 1;
  *n_exchanges = 0;
  *n_local = 0;
  const double sgn = inv ? 1.0 : -1.0;
  for (int S = 0; S < st.n; ++S) {
    const int R = st.r[S];
    const int NB = E / R;
    const bool last = S + 1 == st.n;
    const bool local = tbs::stage_is_local(M, E, S);
    const tbs::Swz xl = tbs::swz_of(M, TPT, L, R, 16);
    for (int t = 0; t < TPT; ++t) {
      for (int q = 0; q < NB; ++q) {
        const int b = t + q * TPT;
        const int k = b % L;
        tbs::cx<double> a[16];
        for (int r = 0; r < R; ++r) {
          a[r] = v[(size_t)t * E + q + r * NB];
          if (S > 0 && r > 0) {
            const double ang = sgn * 2.0 * M_PI * (double)(r * k) / (double)(L * R);
            a[r] = tbs::cmul(a[r], tbs::cx<double>{std::cos(ang), std::sin(ang)});
          }
        }
        if (inv) dft_rt<true>(R, a); else dft_rt<false>(R, a);
        for (int r = 0; r < R; ++r) {
          if (last) w[(size_t)t * E + q + r * NB] = a[r];
          else if (local) w[(size_t)t * E + tbs::local_register(q, r, TPT, L, R)] = a[r];
          else sh[(size_t)tbs::xwrite_slot(xl, TPT, L, R, t, q, r)] = a[r];
        }
      }
    }
    if (!last && !local) {
      for (int t = 0; t < TPT; ++t)
        for (int j = 0; j < E; ++j) w[(size_t)t * E + j] = sh[(size_t)tbs::xread_slot(xl, TPT, t, j)];
      ++*n_exchanges;
    } else if (local) {
      ++*n_local;
    }
    v.swap(w);
    L *= R;
  }
  for (int t = 0; t < TPT; ++t)
    for (int j = 0; j < E; ++j) {
      out[2 * (t + j * TPT)] = v[(size_t)t * E + j].x;
      out[2 * (t + j * TPT) + 1] = v[(size_t)t * E + j].y;
    }
  return 0;
}

// The closed-form LDS slots of the device exchanges against their definition
// lpad(index) for every thread, butterfly and output of every stage that
// exchanges through LDS.  Returns the number of mismatches.
extern "C" int tbs_hostcheck_slots(int M, int E) {
  const tbs::Stages st = tbs::make_stages(M, E);
  if (st.n <= 0 || M % E) return -1;
  const int TPT = M / E;
  int bad = 0;
  for (int t = 0; t < TPT; ++t)
    for (int j = 0; j < E; ++j)
      bad += tbs::read_slot(TPT, t, j) != tbs::lpad(t + j * TPT);
  int L = 1;
  for (int S = 0; S < st.n; ++S) {
    const int R = st.r[S];
    if (S + 1 < st.n && !tbs::stage_is_local(M, E, S))
      for (int t = 0; t < TPT; ++t)
        for (int q = 0; q < E / R; ++q)
          for (int r = 0; r < R; ++r)
            bad += tbs::write_slot(TPT, L, R, t, q, r) !=
                   tbs::lpad(tbs::stage_out_index(t + q * TPT, L, R, r));
    L *= R;
  }
  return bad;
}

// The LDS exchange layouts of a pass block of NL lines (LDS elements of esz
// bytes, one buffer of lds_len slots per line) whose lanes take the lines as
// the passes do: kind 0 (column pass) lane l -> line l mod NL, value index
// l / NL; kind 1 (row pass, 4-value column blocks) lane l -> line (l / 4) mod
// NL, value index (l / (4 NL)) 4 + l mod 4.  "new" is the layout the passes
// use (swz_of), "pad" the padded layout throughout.  Checks for the new
// layout: the closed-form slots equal the layout of the indices they stand
// for, every write slot is inside the line's buffer and taken once per stage,
// every read finds the element it stands for.  Bank model of gfx950's LDS: 32
// banks of 4 bytes, 128 / esz lanes of one instruction served per cycle, an
// access of esz bytes covering esz / 4 consecutive banks; lanes of one group
// on one bank at different addresses cost one extra cycle each.  *cyc_pad /
// *cyc_new: the extra cycles of all exchanges of one block (waves of 64
// lanes).  Returns the number of mismatches.
namespace {
int extra_cycles(const std::vector<int>& addr, int esz) {
  const int G = 128 / esz, words = esz / 4;
  int extra = 0;
  for (size_t g0 = 0; g0 < addr.size(); g0 += (size_t)G) {
    std::vector<std::vector<int>> bank(32);
    for (size_t i = g0; i < g0 + (size_t)G && i < addr.size(); ++i)
      for (int d = 0; d < words; ++d) {
        const int a = addr[i] * words + d;
        auto& b = bank[(size_t)(a % 32)];
        bool seen = false;
        for (int x : b) seen |= (x == a);
        if (!seen) b.push_back(a);
      }
    int worst = 1;
    for (auto& b : bank) worst = (int)b.size() > worst ? (int)b.size() : worst;
    extra += worst - 1;
  }
  return extra;
}
}  // namespace

extern "C" int tbs_hostcheck_xslots(int M, int E, int esz, int NL, int kind, int* cyc_pad, int* cyc_new) {
  const tbs::Stages st = tbs::make_stages(M, E);
  if (st.n <= 0 || M % E || (esz != 4 && esz != 8 && esz != 16) || NL < 1 || (kind != 0 && kind != 1))
    return -1;
  const int TPT = M / E;
  if (kind == 1 && TPT % 4) return -1;
  const int G = 128 / esz;
  const int LDP = tbs::lds_len(M, NL, esz);
  const int len_new = NL * LDP;
  const int nth = NL * TPT;
  std::vector<int> lane_line((size_t)nth), lane_t((size_t)nth);
  for (int l = 0; l < nth; ++l) {
    lane_line[(size_t)l] = kind == 0 ? l % NL : (l / 4) % NL;
    lane_t[(size_t)l] = kind == 0 ? l / NL : (l / (4 * NL)) * 4 + l % 4;
  }
  int bad = 0;
  *cyc_pad = 0;
  *cyc_new = 0;
  auto tally = [&](const std::vector<int>& ap, const std::vector<int>& an) {
    for (size_t w0 = 0; w0 < ap.size(); w0 += 64) {
      const size_t w1 = w0 + 64 < ap.size() ? w0 + 64 : ap.size();
      *cyc_pad += extra_cycles(std::vector<int>(ap.begin() + w0, ap.begin() + w1), esz);
      *cyc_new += extra_cycles(std::vector<int>(an.begin() + w0, an.begin() + w1), esz);
    }
  };
  const tbs::Swz pad{0, -1, 0};
  int L = 1;
  for (int S = 0; S + 1 < st.n; ++S) {
    const int R = st.r[S];
    if (!tbs::stage_is_local(M, E, S)) {
      const tbs::Swz xl = tbs::swz_of(M, TPT, L, R, G);
      std::vector<int> at((size_t)NL * M, -1);  // (line, element) -> buffer slot
      std::vector<int> owner((size_t)len_new, -1);
      for (int q = 0; q < E / R; ++q)
        for (int r = 0; r < R; ++r) {
          std::vector<int> ap, an;
          for (int l = 0; l < nth; ++l) {
            const int ln = lane_line[(size_t)l], t = lane_t[(size_t)l];
            const int e = tbs::stage_out_index(t + q * TPT, L, R, r);
            const int sx = tbs::xwrite_slot(xl, TPT, L, R, t, q, r);
            const int want = xl.nb < 0 ? tbs::write_slot(TPT, L, R, t, q, r) : tbs::swz_apply(e, xl);
            bad += sx != want;
            const int addr = ln * LDP + sx;
            if (sx < 0 || sx >= LDP || addr >= len_new || owner[(size_t)addr] >= 0) {
              ++bad;
              continue;
            }
            owner[(size_t)addr] = e;
            at[(size_t)ln * M + e] = addr;
            ap.push_back(ln * LDP + tbs::xwrite_slot(pad, TPT, L, R, t, q, r));
            an.push_back(addr);
          }
          tally(ap, an);
        }
      for (int j = 0; j < E; ++j) {
        std::vector<int> ap, an;
        for (int l = 0; l < nth; ++l) {
          const int ln = lane_line[(size_t)l], t = lane_t[(size_t)l];
          const int sx = tbs::xread_slot(xl, TPT, t, j);
          const int addr = ln * LDP + sx;
          bad += (addr != at[(size_t)ln * M + t + j * TPT]);
          ap.push_back(ln * LDP + tbs::xread_slot(pad, TPT, t, j));
          an.push_back(addr);
        }
        tally(ap, an);
      }
    }
    L *= R;
  }
  return bad;
}

// The register-resident twiddle factors: for every thread, stage S >= 1,
// butterfly q and input r, the cache slot the transform reads holds (as
// tw_load fills it) the table entry of k = (t + q TPT) mod L, and every slot
// lies inside the cache.  Returns the number of mismatches.
extern "C" int tbs_hostcheck_twcache(int M, int E) {
  const tbs::Stages st = tbs::make_stages(M, E);
  if (st.n <= 0 || M % E) return -1;
  const int TPT = M / E;
  const int size = tbs::tw_cache_size(M, E);
  int bad = 0;
  for (int t = 0; t < TPT; ++t) {
    std::vector<int> cache((size_t)size, -1);
    for (int S = 1; S < st.n; ++S) {  // as tw_load
      const int R = st.r[S], L = tbs::stage_L(M, E, S), OFF = tbs::stage_twoff(M, E, S);
      for (int q = 0; q < tbs::tw_classes(M, E, S); ++q)
        for (int r = 1; r < R; ++r) {
          const int slot = tbs::tw_cache_base(M, E, S) + q * (R - 1) + r - 1;
          if (slot < 0 || slot >= size) { ++bad; continue; }
          cache[(size_t)slot] = OFF + (r - 1) * L + (t + q * TPT) % L;
        }
    }
    for (int S = 1; S < st.n; ++S) {  // as fft_stages reads them
      const int R = st.r[S], L = tbs::stage_L(M, E, S), OFF = tbs::stage_twoff(M, E, S);
      for (int q = 0; q < E / R; ++q)
        for (int r = 1; r < R; ++r) {
          const int slot = tbs::tw_cache_base(M, E, S) + (q % tbs::tw_classes(M, E, S)) * (R - 1) + r - 1;
          const int want = OFF + (r - 1) * L + (t + q * TPT) % L;
          bad += (slot < 0 || slot >= size || cache[(size_t)slot] != want);
        }
    }
  }
  return bad;
}

// The bfloat16 storage of the Kahan compensation: out[i] = the 16-bit pattern
// the device stores for in[i]; back[i] = the value it reads back.
extern "C" void tbs_hostcheck_bf16(const float* in, int n, uint32_t* out, float* back) {
  for (int i = 0; i < n; ++i) {
    out[i] = tbs::bf16_bits(in[i]);
    back[i] = tbs::bf16_value(out[i]);
  }
}

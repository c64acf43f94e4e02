// Streaming passes of the zero-padded Green's-function convolution
// u_{n+1} = G (V u_n), G = F^-1 diag(G^) F (paper Sec. 2.2, Eqs. TBS_1 and
// TBS_algorithm), as HBM-streaming CDNA4 kernels.
//
//  * k_row_pass: one x line per grid row.  Inverse x-FFT of the previous term's
//    spectral row, crop to the physical row (term u_{n-1}), Kahan (FP32) or
//    plain (FP64) p += u, FP64 norm partials, w = V u (conj(V) u for the
//    adjoint, or the pairing sum g += conj(u) P for the gradient), zero-pad,
//    forward x-FFT, store.  The first pass reads the source instead.
//  * k_col_pass: one strided line (y in 2D, y or z in 3D) per column: zero-pad,
//    forward FFT, multiply by the folded spectrum G^ (conj for the adjoint),
//    inverse FFT, crop; or only the forward / inverse half of that.
//
// Every FFT line lives in registers of one thread group (see tbs_fft.hpp);
// LDS is used only for the exchanges between radix stages.  Lines are read
// and written in contiguous kBlock-wide column blocks so that every HBM access
// is a full, coalesced segment.
#pragma once

#include <type_traits>

#include "tbs_bf16.hpp"
#include "tbs_fft.hpp"
#include "tbs_internal.hpp"

// Tuning knobs (compile-time; the defaults are the measured best on MI355X).
#ifndef TBS_E_LONG_F32
#define TBS_E_LONG_F32 16   // values per thread, FP32 lines of 2048+
#endif
#ifndef TBS_E_ODD_MUL_F32
#define TBS_E_ODD_MUL_F32 4  // values per thread / odd radix, FP32 lines 3*2^a >= 384, 5*2^a >= 640
#endif
#ifndef TBS_SPLIT_ODD_E
#define TBS_SPLIT_ODD_E 24   // odd-family lines with this many values per thread split re/im
#endif
#ifndef TBS_SPLIT_MIN
#define TBS_SPLIT_MIN 1000000  // shortest line that exchanges re/im separately
#endif
#ifndef TBS_NR_F32
#define TBS_NR_F32 2        // rows per FP32 row-pass block (lines of 2048+)
#endif
#ifndef TBS_NC_F32
#define TBS_NC_F32 2        // columns per FP32 column-convolution block (<= layout block)
#endif
#ifndef TBS_NR_F64
#define TBS_NR_F64 2        // rows per FP64 row-pass block (lines of 4096)
#endif
#ifndef TBS_NC_F64
#define TBS_NC_F64 2        // columns per FP64 column-convolution block (lines of 2048+)
#endif
#ifndef TBS_TW_RESIDENT
#define TBS_TW_RESIDENT 1   // twiddle factors in registers where they fit
#endif
#ifndef TBS_TW_MIN_M
#define TBS_TW_MIN_M 512    // shortest line that keeps its twiddle factors in registers
#endif
#ifndef TBS_OCC_HINT
#define TBS_OCC_HINT 1      // size each pass's register budget to its LDS occupancy
#endif
#ifndef TBS_PREFETCH
#define TBS_PREFETCH 1      // loads issued with the line's own: 1 row sum + compensation,
#endif                      // 2 row potential, 4 column spectrum
#define TBS_PF_ACC ((TBS_PREFETCH & 1) != 0)
#define TBS_PF_V ((TBS_PREFETCH & 2) != 0)
#define TBS_PF_G ((TBS_PREFETCH & 4) != 0)

namespace tbs {

__device__ __forceinline__ void kahan_add(float& s, float& c, float x) {
#pragma clang fp contract(off)
  const float y = x - c;
  const float t = s + y;
  c = (t - s) - y;
  s = t;
}

// Workgroups are dealt round-robin to the 8 XCDs; give each XCD a contiguous
// range of logical blocks so that neighbours (which share table rows / V rows
// through L2) run on the same XCD.
__device__ __forceinline__ int xcd_block(int bid, int nblk, int on) {
  constexpr int kXcd = 8;
  if (!on || (nblk % kXcd) != 0) return bid;
  return (bid % kXcd) * (nblk / kXcd) + bid / kXcd;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <typename T>
__device__ __forceinline__ double norm2(cx<T> a) {
  return (double)a.x * (double)a.x + (double)a.y * (double)a.y;
}

__device__ __forceinline__ int fold(int k, int m) { return k <= (m >> 1) ? k : m - k; }

// Launch order pairing the mirror images k, n-k (n even): 0, 1, n-1, 2, n-2,
// ..., n/2-1, n/2+1, n/2.  A bijection of [0, n); identity for odd n.
__device__ __forceinline__ int mirror_pair(int l, int n) {
  if ((n & 1) || l == 0) return l;
  if (l == n - 1) return n >> 1;
  const int k = (l + 1) >> 1;
  return (l & 1) ? k : n - k;
}

// Density term div(gamma grad u) at cell (z, y, x) of a 2D (nz = 1) or 3D
// field u (the term of the inhomogeneous wave equation of Sec. 2.1.3 that
// carries the density contrast gamma = (rho_s - rho_f) / rho_s): conservative
// second-order differences per axis with gamma at the half points the mean of
// the two cells, u and gamma zero outside the grid; the axis terms are added
// x, y, z in that order.  i: index of the cell in u, c = u(z, y, x).  FP64
// arithmetic.
template <typename T>
__device__ __forceinline__ cx<T> density_term(const RowArgs& a, const void* u,
                                              int64_t i, int z, int y, int x, cx<T> c) {
  const double* g = a.gamma;
  const int64_t sy = a.nx, sz = (int64_t)a.nx * a.ny;
  const int64_t gi = ((int64_t)z * a.ny + y) * a.nx + x;
  const double gc = gld1<double>(g, gi);
  const bool xp = x + 1 < a.nx, xm = x > 0, yp = y + 1 < a.ny, ym = y > 0;
  const bool zp = z + 1 < a.nz, zm = z > 0;
  const double gxp = 0.5 * (gc + (xp ? gld1<double>(g, gi + 1) : 0.0));
  const double gxm = 0.5 * (gc + (xm ? gld1<double>(g, gi - 1) : 0.0));
  const double gyp = 0.5 * (gc + (yp ? gld1<double>(g, gi + sy) : 0.0));
  const double gym = 0.5 * (gc + (ym ? gld1<double>(g, gi - sy) : 0.0));
  const double gzp = a.nz > 1 ? 0.5 * (gc + (zp ? gld1<double>(g, gi + sz) : 0.0)) : 0.0;
  const double gzm = a.nz > 1 ? 0.5 * (gc + (zm ? gld1<double>(g, gi - sz) : 0.0)) : 0.0;
  if (gxp == 0.0 && gxm == 0.0 && gyp == 0.0 && gym == 0.0 && gzp == 0.0 && gzm == 0.0)
    return cx<T>{T(0), T(0)};
  const cx<T> zero = {T(0), T(0)};
  const cx<T> uxp = xp ? gld<T>(u, i + 1) : zero, uxm = xm ? gld<T>(u, i - 1) : zero;
  const cx<T> uyp = yp ? gld<T>(u, i + sy) : zero, uym = ym ? gld<T>(u, i - sy) : zero;
  const double cr = c.x, ci = c.y;
  double re = gxp * ((double)uxp.x - cr) - gxm * (cr - (double)uxm.x);
  double im = gxp * ((double)uxp.y - ci) - gxm * (ci - (double)uxm.y);
  re += gyp * ((double)uyp.x - cr) - gym * (cr - (double)uym.x);
  im += gyp * ((double)uyp.y - ci) - gym * (ci - (double)uym.y);
  if (a.nz > 1) {
    const cx<T> uzp = zp ? gld<T>(u, i + sz) : zero, uzm = zm ? gld<T>(u, i - sz) : zero;
    re += gzp * ((double)uzp.x - cr) - gzm * (cr - (double)uzm.x);
    im += gzp * ((double)uzp.y - ci) - gzm * (ci - (double)uzm.y);
  }
  return cx<T>{(T)(re * a.inv_dx2), (T)(im * a.inv_dx2)};
}

// Waves on the fullest SIMD of a CU when the LDS of one block (LINES lines
// of length M; 160 KB per CU, 4 SIMDs, at most 8 waves each) limits the
// blocks a CU holds.
template <typename T>
constexpr int lds_only_waves(int M, int E, int lines, bool split) {
  const int esz = split ? (int)sizeof(T) : 2 * (int)sizeof(T);
  const long lds = (long)lines * lds_len(M, lines, esz) * esz;
  const int waves_blk = (lines * (M / E) + 63) / 64;
  long blocks = (160L * 1024) / lds;
  if (blocks * waves_blk > 32) blocks = 32 / waves_blk;
  const int w = (int)((blocks * waves_blk + 3) / 4);  // the fullest SIMD
  return w < 1 ? 1 : w;
}

// Whether a pass keeps the twiddle factors of its transforms in registers
// (loaded once, shared by its forward and inverse transform): lines of
// TBS_TW_MIN_M and more, when the E values and the factors (2 VGPRs per FP32
// complex, 4 per FP64) plus the rest of the pass fit the registers that the
// LDS occupancy leaves the waves of the fullest SIMD, or at most 128 VGPRs
// (256 in FP64) where that is more: fewer loads beat the occupancy they cost
// (the 3D z convolution at 512 ran 18 % faster with the factors at 6 waves per
// SIMD than without them at 8; its FP64 version 15 % faster).  The rest (FP32;
// twice in FP64) is what the compiled kernels take: about 32 VGPRs in the
// column pass and 40 in the row pass (48 at 512) for power-of-two lines, 80
// and 72 for lines with a radix-3 or radix-5 stage.  With these margins no
// kernel spills more than one register, except two FP32 2048 column kernels
// with the uniform loads of col_pass_body (2 and 6 registers; still the faster
// variant).  The forward-only column pass (3D y) keeps loading from the
// table: it runs one transform, and the lower occupancy made it 5 % slower.
// The choice is made per length and pass, at the pass's default block shape
// (rows_per_block; conv_default_cols), and holds for every block shape of
// that length: where the factors come from changes how the compiler fuses the
// products of the odd-radix butterflies (results then differ in the last
// bits), so one choice per length keeps the block-shape candidates of the
// autotuners bitwise-neutral.  FP32 column passes of 3 * 2^a lines keep the
// factors in registers beyond the estimate (126 VGPRs at two lines per block,
// 4 waves per SIMD, no spills; the 1536 column convolution of the broadband
// batch 22.3 -> 18.0 ms per step; their row passes ran 34 % slower with
// them), those of 5 * 2^a lines load them from the table (the tuned 1280 and
// 2560 convolutions of that batch, 2 and 1 lines per block, ran 6 % and 1 %
// slower with them in registers; FP64 as well: the batch 962 -> 914 ms/step).
constexpr int rows_per_block(int M, bool fp64);
constexpr int conv_default_cols(int M, bool fp64);
template <typename T>
constexpr int tw_resident_vgprs(int M, int E, bool row) {
  const bool odd = (M & (M - 1)) != 0;
  const int rest = odd ? (row ? 72 : 80) : (row ? (M <= 512 ? 48 : 40) : 32);
  // early-issued loads held in registers across the first transform: per
  // value of the first half of the line the sum, its compensation and the
  // potential (row pass; 5 VGPRs in FP32, 8 in FP64), or per value the
  // spectrum (column pass)
  const int pre = row ? (E / 2) * ((TBS_PF_ACC ? (sizeof(T) == 4 ? 3 : 4) : 0) + (TBS_PF_V ? (int)(sizeof(T) / 2) : 0))
                      : ((TBS_PF_G || (sizeof(T) == 8 && E <= 8)) ? E * (int)(sizeof(T) / 2) : 0);
  return (int)(sizeof(T) / 2) * (E + tw_cache_size(M, E)) + rest * (int)(sizeof(T) / 4) + pre;
}
template <typename T>
constexpr bool tw_resident(int M, int E, bool split, bool row) {
  constexpr bool F64 = sizeof(T) == 8;
  if (!F64 && !row && M % 3 == 0) return TBS_TW_RESIDENT && M >= TBS_TW_MIN_M;
  if (!row && M % 5 == 0) return false;
  const int lines = row ? rows_per_block(M, F64) : conv_default_cols(M, F64);
  const int budget = 512 / lds_only_waves<T>(M, E, lines, split);
  const int block_waves_simd = (lines * (M / E) + 255) / 256;  // a block's waves share 4 SIMDs
  const int floor_regs = 128 * (int)(sizeof(T) / 4) < 512 / block_waves_simd
                             ? 128 * (int)(sizeof(T) / 4) : 512 / block_waves_simd;
  return TBS_TW_RESIDENT && M >= TBS_TW_MIN_M &&
         tw_resident_vgprs<T>(M, E, row) <= (budget > floor_regs ? budget : floor_regs);
}

// Resident waves per SIMD a pass asks the compiler to budget registers for
// (512 VGPRs per SIMD lane, shared by its waves): what the LDS allows, but no
// more than a line of E values per thread can keep in registers without
// spilling (about 5 E + 40 VGPRs in FP32, twice the values in FP64, at least
// 112; with resident twiddles the estimate above).  Without the request,
// lines of 40 values per thread compiled to more than 256 VGPRs: one wave per
// SIMD.
// KIND: 0 a kernel without resident twiddles, 1 the row pass, 2 the column pass.
template <typename T, int KIND>
constexpr int lds_waves_per_eu(int M, int E, int lines, bool split) {
  if (!TBS_OCC_HINT) return 1;
  int w = lds_only_waves<T>(M, E, lines, split);
  const int need = (sizeof(T) == 8 ? 10 : 5) * E + 40;
  const int regs = (KIND != 0 && tw_resident<T>(M, E, split, KIND == 1))
                       ? tw_resident_vgprs<T>(M, E, KIND == 1)
                       : (need < 112 ? 112 : need);
  const int wr = 512 / regs;
  if (w > wr) w = wr;
  return w < 1 ? 1 : (w > 8 ? 8 : w);
}

#define TBS_OCCUPANCY(T, M, E, LINES, SPLIT, KIND) \
  __attribute__((amdgpu_waves_per_eu(lds_waves_per_eu<T, KIND>(M, E, LINES, SPLIT), 8)))

// ---------------------------------------------------------------- row pass --

template <typename T, int M, int E, int NR, int CB, bool SPLIT>
__device__ __forceinline__ void row_pass_body(const RowArgs& a, const int lb) {
  constexpr int TPT = M / E;
  constexpr int NKB = M / CB;
  constexpr int LD = lds_len(M, NR, SPLIT ? sizeof(T) : 2 * sizeof(T));
  constexpr int NT = NR * TPT;
  constexpr int NW = (NT + 63) / 64;
  static_assert(TPT % CB == 0, "line too short for the column block");
  static_assert(E % 2 == 0, "E must be even");
  using LdsT = typename std::conditional<SPLIT, T, cx<T>>::type;
  __shared__ LdsT sh[NR * LD];
  __shared__ double red[2 * NW];

  const int tid = threadIdx.x;
  const int tlo = tid % CB;
  const int r = (tid / CB) % NR;
  const int thi = tid / (CB * NR);
  const int t = thi * CB + tlo;
  const int rhs = lb % a.nrhs;
  const int rb = lb / a.nrhs;
  const int nblk = (a.nrows + NR - 1) / NR;
  const int row = rb * NR + r;
  const bool valid = row < a.nrows;
  LdsT* shr = sh + r * LD;
  const cx<T>* tw = (const cx<T>*)a.tw;
  void* X = a.X;
  const int64_t P = (int64_t)a.nrows * a.nx;
  const int yy = valid ? row / a.nz : 0;
  const int zz = valid ? row % a.nz : 0;
  const int64_t srow = (int64_t)(zz * a.ny + yy) * a.nx;  // spatial offset of this row
  const int64_t sp_base = (int64_t)rhs * P + srow;
  const int64_t xbase = ((int64_t)rhs * NKB * a.nrows + (valid ? row : 0)) * CB;
  const int64_t kbstride = (int64_t)a.nrows * CB;

  cx<T> v[E];
  constexpr bool TWR = tw_resident<T>(M, E, SPLIT, true);
  cx<T> twc[TWR ? tw_cache_size(M, E) : 1];
  if constexpr (TWR) tw_load<T, M, E>(twc, tw, t);
  double su = 0.0, sp = 0.0;
  if (a.in_mode == ROW_IN_SPECTRAL) {
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int kx = t + j * TPT;
      v[j] = valid ? gld<T>(X, xbase + (int64_t)(kx / CB) * kbstride + (kx % CB)) : cx<T>{T(0), T(0)};
    }
    void* p = a.p;
    const void* Vp = a.V;
    // The sum, its compensation and the potential of this row do not depend
    // on the transform: their loads can be issued with the spectrum's, so
    // that their latency overlaps the inverse FFT (TBS_PREFETCH).
    constexpr int EA = TBS_PF_ACC ? E / 2 : 1;
    constexpr int EV = TBS_PF_V ? E / 2 : 1;
    cx<T> pre_p[EA], pre_v[EV];
    uint32_t pre_c[EA];
    if constexpr (TBS_PF_ACC) {
      const bool pf = a.acc == ACC_ADD;
#pragma unroll
      for (int j = 0; j < EA; ++j) {
        const int x = t + j * TPT;
        const bool in = pf && valid && x < a.nx;
        pre_p[j] = in ? gld<T>(p, sp_base + x) : cx<T>{T(0), T(0)};
        pre_c[j] = (sizeof(T) == 4 && in) ? gld1<uint32_t>(a.c, sp_base + x) : 0u;
      }
    }
    if constexpr (TBS_PF_V) {
      const bool pf = a.out_spec && Vp != nullptr;
#pragma unroll
      for (int j = 0; j < EV; ++j) {
        const int x = t + j * TPT;
        pre_v[j] = (pf && valid && x < a.nx) ? gld<T>(Vp, srow + x) : cx<T>{T(0), T(0)};
      }
    }
    if constexpr (TWR) fft_cached<T, M, E, true, SPLIT>(v, shr, twc, t);
    else fft<T, M, E, true, SPLIT>(v, shr, tw, t);
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int x = t + j * TPT;
      cx<T> w = {T(0), T(0)};
      if (j < E / 2 && valid && x < a.nx) {
        const int64_t i = sp_base + x;
        const cx<T> u = v[j];
        if (a.ustore) gst<T>(a.ustore, i, u);
        if (a.acc == ACC_INIT) {
          gst<T>(p, i, u);
          if (a.pstore) gst<T>(a.pstore, i, u);
          if constexpr (sizeof(T) == 4) gst1<uint32_t>(a.c, i, 0u);
          const double n = norm2(u);
          su += n;
          sp += n;
        } else if (a.acc == ACC_ADD) {
          cx<T> pp = TBS_PF_ACC ? pre_p[j % EA] : gld<T>(p, i);
          if constexpr (sizeof(T) == 4) {
            cx<T> ci;
            bf16_unpack(TBS_PF_ACC ? pre_c[j % EA] : gld1<uint32_t>(a.c, i), ci.x, ci.y);
            kahan_add(pp.x, ci.x, u.x);
            kahan_add(pp.y, ci.y, u.y);
            gst1<uint32_t>(a.c, i, bf16_pack(ci.x, ci.y));
          } else {
            pp = pp + u;
          }
          gst<T>(p, i, pp);
          if (a.pstore) gst<T>(a.pstore, i, pp);
          su += norm2(u);
          sp += norm2(pp);
        } else if (a.acc == ACC_PAIR) {
          const cx<T> pr = gld<T>(a.pair, i);
          gst<T>(a.grad, i, gld<T>(a.grad, i) + cmulc(pr, u));   // conj(u) * P
          su += norm2(u);
        }
        if (a.out_spec && Vp != nullptr) {
          const cx<T> vv = TBS_PF_V ? pre_v[j % EV] : gld<T>(Vp, srow + x);
          w = a.conj_v ? cmulc(u, vv) : cmul(u, vv);
        }
      }
      v[j] = w;
    }
  } else {
    const void* src = a.src;
    const void* Vp = a.V;
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int x = t + j * TPT;
      cx<T> w = {T(0), T(0)};
      if (j < E / 2 && valid && x < a.nx) {
        w = gld<T>(src, sp_base + x);
        if (a.in_mode == ROW_IN_SPATIAL) {
          const cx<T> u0 = w;
          if (Vp != nullptr) {
            const cx<T> vv = gld<T>(Vp, srow + x);
            w = a.conj_v ? cmulc(w, vv) : cmul(w, vv);
          } else {
            w = cx<T>{T(0), T(0)};
          }
          if (a.gamma != nullptr) w = w - density_term<T>(a, src, sp_base + x, zz, yy, x, u0);
        }
      }
      v[j] = w;
    }
  }

  if (a.acc != ACC_NONE) {
    su = wave_sum(su);
    sp = wave_sum(sp);
    const int wv = tid >> 6;
    if ((tid & 63) == 0) {
      red[2 * wv] = su;
      red[2 * wv + 1] = sp;
    }
    __syncthreads();
    if (tid == 0) {
      // every thread of the block works on rows of the same rhs
      double a0 = 0.0, a1 = 0.0;
      for (int k = 0; k < NW; ++k) {
        a0 += red[2 * k];
        a1 += red[2 * k + 1];
      }
      gst1<double>(a.partials, 2 * ((int64_t)rhs * nblk + rb), a0);
      gst1<double>(a.partials, 2 * ((int64_t)rhs * nblk + rb) + 1, a1);
    }
  }

  if (a.out_spec) {  // registers j >= E/2 hold zeros (the padding)
    if constexpr (TWR) fft_cached<T, M, E, false, SPLIT, true>(v, shr, twc, t);
    else fft<T, M, E, false, SPLIT, true>(v, shr, tw, t);
    if (valid) {
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const int kx = t + j * TPT;
        gst<T>(X, xbase + (int64_t)(kx / CB) * kbstride + (kx % CB), v[j]);
      }
    }
  }
}

// ------------------------------------------------------------- column pass --

template <typename T, int M, int E, int NC, int OP, bool SPLIT>
__device__ __forceinline__ void col_pass_body(const ColArgs& a, const int lb) {
  constexpr int TPT = M / E;
  constexpr int LD = lds_len(M, NC, SPLIT ? sizeof(T) : 2 * sizeof(T));
  constexpr bool HALF_IN = (OP == COL_CONV || OP == COL_FWD);
  constexpr bool HALF_OUT = (OP == COL_CONV || OP == COL_INV);
  constexpr bool CONV = (OP == COL_CONV || OP == COL_CONV_FULL);
  using LdsT = typename std::conditional<SPLIT, T, cx<T>>::type;
  __shared__ LdsT sh[NC * LD];

  const int tid = threadIdx.x;
  const int col = tid % NC;
  const int tt = tid / NC;
  const int rhs = lb % a.nrhs;
  const int rest = lb / a.nrhs;
  int i0 = rest % a.n0;
  int i1 = rest / a.n0;
  if (a.mirror) {
    // neighbours in launch order read the same folded spectrum lines
    i0 = mirror_pair(i0, a.n0);
    i1 = mirror_pair(i1 / a.sub, a.n1 / a.sub) * a.sub + i1 % a.sub;
  }
  const bool cvalid = (i0 * a.zcols + col / a.cb) < a.zlim;
  LdsT* shc = sh + col * LD;
  const cx<T>* tw = (const cx<T>*)a.tw;
  const void* in = a.in;
  void* out = a.out;
  // a.sub > 1: the block holds NC of the cb columns of layout block i1 / sub
  const int blk = i1 / a.sub;
  const int c0 = (i1 % a.sub) * NC;
  const int64_t ib = rhs * a.in_rs + blk * a.in_s1 + i0 * a.in_s0 + c0 + col;
  const int64_t ob = rhs * a.out_rs + blk * a.out_s1 + i0 * a.out_s0 + c0 + col;

  cx<T> v[E];
  constexpr bool TWR = OP != COL_CONV_FULL && OP != COL_FWD && tw_resident<T>(M, E, SPLIT, false);
  cx<T> twc[TWR ? tw_cache_size(M, E) : 1];
  constexpr int NLD = HALF_IN ? E / 2 : E;  // registers that can hold input
  // FP32 lines of 2048+: when every position of those registers is inside
  // the line (the usual case, N = M / 2), the same loads without per-lane
  // selects (shorter lines and FP64 ran slower with the second code path)
  constexpr bool UNIFORM = sizeof(T) == 4 && M >= 2048;
  if (UNIFORM && cvalid && a.n_in >= NLD * TPT) {
#pragma unroll
    for (int j = 0; j < E; ++j)
      v[j] = j < NLD ? gld<T>(in, ib + (tt + j * TPT) * a.in_astride) : cx<T>{T(0), T(0)};
  } else {
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int pos = tt + j * TPT;
      const bool ld = j < NLD && cvalid && pos < a.n_in;
      v[j] = ld ? gld<T>(in, ib + pos * a.in_astride) : cx<T>{T(0), T(0)};
    }
  }
  if constexpr (TWR) tw_load<T, M, E>(twc, tw, tt);
  // the spectrum values of this line, loaded with the line (TBS_PREFETCH) so
  // that their latency overlaps the forward FFT
  // (always for FP64 lines of 8 values per thread or fewer: with the 3D z
  // convolution at 512 the FP64 harmonic3d step ran 86.7 -> 81.5 ms; the
  // FP32 one lost a wave per SIMD to the registers and ran 0.4 % slower)
  constexpr bool PFG = TBS_PF_G || (sizeof(T) == 8 && E <= 8);
  constexpr int EG = (CONV && PFG) ? E : 1;
  cx<T> pre_g[EG];
  int64_t gb = 0;
  if constexpr (CONV) {
    const int kx = blk * a.cb + c0 + (col % a.cb);
    gb = fold(kx, a.mx) * a.g_sx + fold(i0, a.mm) * a.g_sm;
    if constexpr (PFG) {
#pragma unroll
      for (int j = 0; j < E; ++j) pre_g[j] = gld<T>(a.ghat, gb + fold(tt + j * TPT, M));
    }
  }
  if constexpr (OP != COL_INV) {
    if constexpr (TWR) fft_cached<T, M, E, false, SPLIT, HALF_IN>(v, shc, twc, tt);
    else fft<T, M, E, false, SPLIT, HALF_IN>(v, shc, tw, tt);
  }
  if constexpr (CONV) {
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const cx<T> gv = PFG ? pre_g[j % EG] : gld<T>(a.ghat, gb + fold(tt + j * TPT, M));
      v[j] = a.conj_g ? cmulc(v[j], gv) : cmul(v[j], gv);
    }
  }
  if constexpr (CONV || OP == COL_INV) {
    if constexpr (TWR) fft_cached<T, M, E, true, SPLIT>(v, shc, twc, tt);
    else fft<T, M, E, true, SPLIT>(v, shc, tw, tt);
  }
  constexpr int NST = HALF_OUT ? E / 2 : E;  // registers that can hold output
  if (UNIFORM && cvalid && a.n_out >= NST * TPT) {
#pragma unroll
    for (int j = 0; j < NST; ++j) gst<T>(out, ob + (tt + j * TPT) * a.out_astride, v[j]);
  } else if (cvalid) {
#pragma unroll
    for (int j = 0; j < NST; ++j) {
      const int pos = tt + j * TPT;
      if (pos < a.n_out) gst<T>(out, ob + pos * a.out_astride, v[j]);
    }
  }
}

// Plain in-place FFT of contiguous rows [nrows][M] (tabulation, FP64).
template <typename T, int M, int E, int NR, bool SPLIT>
__global__ void __launch_bounds__(NR * (M / E)) TBS_OCCUPANCY(T, M, E, NR, SPLIT, 0) k_row_fft_full(cx<T>* data, const cx<T>* tw,
                                                               int nrows, int inverse) {
  constexpr int TPT = M / E;
  constexpr int LD = lds_len(M, NR, SPLIT ? sizeof(T) : 2 * sizeof(T));
  using LdsT = typename std::conditional<SPLIT, T, cx<T>>::type;
  __shared__ LdsT sh[NR * LD];
  const int tid = threadIdx.x;
  const int r = tid / TPT;
  const int t = tid % TPT;
  const int row = blockIdx.x * NR + r;
  const bool valid = row < nrows;
  cx<T>* d = data + (int64_t)(valid ? row : 0) * M;
  cx<T> v[E];
#pragma unroll
  for (int j = 0; j < E; ++j) v[j] = valid ? d[t + j * TPT] : cx<T>{T(0), T(0)};
  if (inverse)
    fft<T, M, E, true, SPLIT>(v, sh + r * LD, tw, t);
  else
    fft<T, M, E, false, SPLIT>(v, sh + r * LD, tw, t);
  if (valid) {
#pragma unroll
    for (int j = 0; j < E; ++j) d[t + j * TPT] = v[j];
  }
}

// ---------------------------------------------------------------- kernels --

template <typename T, int M, int E, int NR, int CB, bool SPLIT>
__global__ void __launch_bounds__(NR * (M / E)) TBS_OCCUPANCY(T, M, E, NR, SPLIT, 1) k_row_pass(RowArgs a) {
  row_pass_body<T, M, E, NR, CB, SPLIT>(a, xcd_block(blockIdx.x, gridDim.x, a.xcd_remap));
}

template <typename T, int M, int E, int NC, int OP, bool SPLIT>
__global__ void __launch_bounds__(NC * (M / E)) TBS_OCCUPANCY(T, M, E, NC, SPLIT, OP == COL_FWD ? 0 : 2) k_col_pass(ColArgs a) {
  col_pass_body<T, M, E, NC, OP, SPLIT>(a, xcd_block(blockIdx.x, gridDim.x, a.xcd_remap));
}

// Grouped launches: one kernel for several grids with the same line length.
// Grid g owns blocks [starts[g], starts[g+1]); its arguments are descs[g].
__device__ __forceinline__ int group_of(const int* __restrict__ starts, int ngroups, int b) {
  int g = 0;
  while (g + 1 < ngroups && starts[g + 1] <= b) ++g;
  return g;
}

template <typename T, int M, int E, int NR, int CB, bool SPLIT>
__global__ void __launch_bounds__(NR * (M / E)) TBS_OCCUPANCY(T, M, E, NR, SPLIT, 1)
    k_row_pass_group(const RowArgs* __restrict__ descs,
                                                                 const int* __restrict__ starts,
                                                                 int ngroups) {
  const int b = xcd_block(blockIdx.x, gridDim.x, 1);
  const int g = group_of(starts, ngroups, b);
  row_pass_body<T, M, E, NR, CB, SPLIT>(descs[g], b - starts[g]);
}

template <typename T, int M, int E, int NC, int OP, bool SPLIT>
__global__ void __launch_bounds__(NC * (M / E)) TBS_OCCUPANCY(T, M, E, NC, SPLIT, OP == COL_FWD ? 0 : 2)
    k_col_pass_group(const ColArgs* __restrict__ descs,
                                                                 const int* __restrict__ starts,
                                                                 int ngroups) {
  const int b = xcd_block(blockIdx.x, gridDim.x, 1);
  const int g = group_of(starts, ngroups, b);
  col_pass_body<T, M, E, NC, OP, SPLIT>(descs[g], b - starts[g]);
}

// ------------------------------------------------------- configurations ---

// Odd part of a length (1, 3 or 5 for the compiled families).
constexpr int odd_part(int M) {
  while (M % 2 == 0) M /= 2;
  return M;
}

// Values per thread.  Powers of two: 4 / 8 / 16 by length (FP32 lines of
// 2048+ use TBS_E_LONG_F32).  3 * 2^a and 5 * 2^a: 4 * odd part (radix-4
// stages, one radix-2 if needed, one odd stage); FP32 lines of 384+ / 640+
// use TBS_E_ODD_MUL_F32 * odd part (8: radix-8 stages, fewer exchanges but
// twice the registers and one wave per line).
constexpr int elems_per_thread(int M, bool fp64) {
  const int r = odd_part(M);
  if (r == 1) return M <= 64 ? 4 : (M <= 512 ? 8 : ((M <= 1024 || fp64) ? 16 : TBS_E_LONG_F32));
  if (!fp64 && ((r == 3 && M >= 384) || (r == 5 && M >= 640))) return TBS_E_ODD_MUL_F32 * r;
  return 4 * r;
}
// Exchanges split into real and imaginary rounds (half the LDS per line) for
// lines whose many values per thread would otherwise leave few lines per CU.
constexpr bool split_lds(int M, bool fp64) {
  return M >= TBS_SPLIT_MIN || (odd_part(M) > 1 && elems_per_thread(M, fp64) >= TBS_SPLIT_ODD_E);
}
constexpr int rows_per_block(int M, bool fp64) {
  return fp64 ? (M >= 4096 ? TBS_NR_F64 : (M >= 2048 && !split_lds(M, true) ? 2 : 4))
              : (M >= 2048 ? TBS_NR_F32 : 4);
}
// Columns per convolution block with a layout block of 4 columns (the
// default of conv_cols_per_block).
constexpr int conv_default_cols(int M, bool fp64) { return M >= 2048 ? (fp64 ? TBS_NC_F64 : TBS_NC_F32) : 4; }
constexpr bool col_fits(int M, int NC, int esz) {
  const int le = split_lds(M, esz == 16) ? esz / 2 : esz;
  return (long)NC * lds_len(M, NC, le) * le <= 160L * 1024;
}

// ------------------------------------------------------ launch templates --

constexpr bool row_fits(int M, int NR, int esz) {
  const int le = split_lds(M, esz == 16) ? esz / 2 : esz;
  return (long)NR * lds_len(M, NR, le) * le <= 160L * 1024;
}

// Row-pass block shapes: the default NR, or (lines of 2048+) 2 or 4 rows when
// they fit LDS; nr = 0 selects the default.
template <typename T, int M, int NR>
int row_launch_nr(const RowArgs& a, int nblk_rows, hipStream_t s) {
  constexpr bool F64 = sizeof(T) == 8;
  constexpr int E = elems_per_thread(M, F64);
  constexpr bool SP = split_lds(M, F64);
  const int grid = nblk_rows * a.nrhs;
  if (a.cb == 4) {
    hipLaunchKernelGGL((k_row_pass<T, M, E, NR, 4, SP>), dim3(grid), dim3(NR * (M / E)), 0, s, a);
  } else if (a.cb == 2) {
    hipLaunchKernelGGL((k_row_pass<T, M, E, NR, 2, SP>), dim3(grid), dim3(NR * (M / E)), 0, s, a);
  } else {
    return (int)hipErrorInvalidValue;
  }
  return (int)hipGetLastError();
}

template <typename T, int M>
int row_launch(const RowArgs& a, int nblk_rows, int nr, hipStream_t s) {
  constexpr bool F64 = sizeof(T) == 8;
  constexpr int NRD = rows_per_block(M, F64);
  constexpr int esz = (int)sizeof(cx<T>);
  if (nr == 0 || nr == NRD) return row_launch_nr<T, M, NRD>(a, nblk_rows, s);
  if constexpr (M >= 2048 && NRD != 2 && row_fits(M, 2, esz)) {
    if (nr == 2) return row_launch_nr<T, M, 2>(a, nblk_rows, s);
  }
  if constexpr (M >= 2048 && NRD != 4 && row_fits(M, 4, esz)) {
    if (nr == 4) return row_launch_nr<T, M, 4>(a, nblk_rows, s);
  }
  return (int)hipErrorInvalidValue;
}

template <typename T, int M, int NR>
int row_group_launch_nr(const RowArgs* descs, const int* starts, int ngroups, int total, int cb,
                        hipStream_t s) {
  constexpr bool F64 = sizeof(T) == 8;
  constexpr int E = elems_per_thread(M, F64);
  constexpr bool SP = split_lds(M, F64);
  if (cb == 4) {
    hipLaunchKernelGGL((k_row_pass_group<T, M, E, NR, 4, SP>), dim3(total), dim3(NR * (M / E)), 0, s,
                       descs, starts, ngroups);
  } else if (cb == 2) {
    hipLaunchKernelGGL((k_row_pass_group<T, M, E, NR, 2, SP>), dim3(total), dim3(NR * (M / E)), 0, s,
                       descs, starts, ngroups);
  } else {
    return (int)hipErrorInvalidValue;
  }
  return (int)hipGetLastError();
}

template <typename T, int M>
int row_group_launch(const RowArgs* descs, const int* starts, int ngroups, int total, int cb, int nr,
                     hipStream_t s) {
  constexpr bool F64 = sizeof(T) == 8;
  constexpr int NRD = rows_per_block(M, F64);
  constexpr int esz = (int)sizeof(cx<T>);
  if (nr == 0 || nr == NRD) return row_group_launch_nr<T, M, NRD>(descs, starts, ngroups, total, cb, s);
  if constexpr (M >= 2048 && NRD != 2 && row_fits(M, 2, esz)) {
    if (nr == 2) return row_group_launch_nr<T, M, 2>(descs, starts, ngroups, total, cb, s);
  }
  if constexpr (M >= 2048 && NRD != 4 && row_fits(M, 4, esz)) {
    if (nr == 4) return row_group_launch_nr<T, M, 4>(descs, starts, ngroups, total, cb, s);
  }
  return (int)hipErrorInvalidValue;
}

template <typename T, int M, int NC>
int col_launch(const ColArgs& a, hipStream_t s) {
  constexpr int E = elems_per_thread(M, sizeof(T) == 8);
  constexpr bool SP = split_lds(M, sizeof(T) == 8);
  const int grid = a.nrhs * a.n1 * a.n0;
  const dim3 blk(NC * (M / E));
  switch (a.op) {
    case COL_CONV:
      hipLaunchKernelGGL((k_col_pass<T, M, E, NC, COL_CONV, SP>), dim3(grid), blk, 0, s, a);
      break;
    case COL_FWD:
      hipLaunchKernelGGL((k_col_pass<T, M, E, NC, COL_FWD, SP>), dim3(grid), blk, 0, s, a);
      break;
    case COL_INV:
      hipLaunchKernelGGL((k_col_pass<T, M, E, NC, COL_INV, SP>), dim3(grid), blk, 0, s, a);
      break;
    default:
      if constexpr (sizeof(T) == 8) {
        hipLaunchKernelGGL((k_col_pass<T, M, E, NC, COL_FULL, SP>), dim3(grid), blk, 0, s, a);
      } else {
        return (int)hipErrorInvalidValue;
      }
  }
  return (int)hipGetLastError();
}

template <typename T, int M>
int col_launch_nc(int NC, const ColArgs& a, hipStream_t s) {
  constexpr int esz = (int)sizeof(cx<T>);
  if constexpr (col_fits(M, 4, esz)) {
    if (NC == 4) return col_launch<T, M, 4>(a, s);
  }
  if constexpr (col_fits(M, 2, esz)) {
    if (NC == 2) return col_launch<T, M, 2>(a, s);
  }
  if constexpr (M >= 2048) {
    if (NC == 1) return col_launch<T, M, 1>(a, s);
  }
  if constexpr (M <= 512 && col_fits(M, 16, esz)) {
    if (NC == 16) return col_launch<T, M, 16>(a, s);
  }
  return (int)hipErrorInvalidValue;
}

// Grouped convolution passes (2D column convolution only).
template <typename T, int M>
int col_group_launch(int NC, const ColArgs* descs, const int* starts, int ngroups, int total,
                     hipStream_t s) {
  constexpr int E = elems_per_thread(M, sizeof(T) == 8);
  constexpr bool SP = split_lds(M, sizeof(T) == 8);
  constexpr int esz = (int)sizeof(cx<T>);
  if constexpr (col_fits(M, 4, esz)) {
    if (NC == 4) {
      hipLaunchKernelGGL((k_col_pass_group<T, M, E, 4, COL_CONV, SP>), dim3(total), dim3(4 * (M / E)),
                         0, s, descs, starts, ngroups);
      return (int)hipGetLastError();
    }
  }
  if constexpr (col_fits(M, 2, esz)) {
    if (NC == 2) {
      hipLaunchKernelGGL((k_col_pass_group<T, M, E, 2, COL_CONV, SP>), dim3(total), dim3(2 * (M / E)),
                         0, s, descs, starts, ngroups);
      return (int)hipGetLastError();
    }
  }
  if constexpr (M >= 2048) {
    if (NC == 1) {
      hipLaunchKernelGGL((k_col_pass_group<T, M, E, 1, COL_CONV, SP>), dim3(total), dim3(M / E), 0, s,
                         descs, starts, ngroups);
      return (int)hipGetLastError();
    }
  }
  return (int)hipErrorInvalidValue;
}

template <int M>
int rowfull_launch(void* data, const void* tw, int nrows, int inverse, hipStream_t s) {
  constexpr int E = elems_per_thread(M, true);
  constexpr int NR = rows_per_block(M, true);
  hipLaunchKernelGGL((k_row_fft_full<double, M, E, NR, split_lds(M, true)>), dim3((nrows + NR - 1) / NR),
                     dim3(NR * (M / E)), 0, s, (cx<double>*)data, (const cx<double>*)tw, nrows,
                     inverse);
  return (int)hipGetLastError();
}

// One family of lengths: dispatches every launch kind for the lengths of its
// list; returns hipErrorInvalidValue for a length it does not hold.
#define TBS_FAMILY_DISPATCH(NAME, LIST)                                                          \
  int NAME(const PassReq& q, hipStream_t s) {                                                    \
    switch (q.M) {                                                                               \
      LIST(TBS_FAMILY_CASE)                                                                       \
      default:                                                                                    \
        return (int)hipErrorInvalidValue;                                                         \
    }                                                                                             \
  }
#define TBS_FAMILY_CASE(m)                                                                        \
  case m:                                                                                         \
    switch (q.kind) {                                                                             \
      case PASS_ROW:                                                                              \
        return q.fp64 ? row_launch<double, m>(*q.row, q.nblk_rows, q.nr, s)                       \
                      : row_launch<float, m>(*q.row, q.nblk_rows, q.nr, s);                       \
      case PASS_COL:                                                                              \
        return q.fp64 ? col_launch_nc<double, m>(q.nc, *q.col, s)                                 \
                      : col_launch_nc<float, m>(q.nc, *q.col, s);                                 \
      case PASS_ROW_FULL:                                                                         \
        return rowfull_launch<m>(q.data, q.tw, q.nrows, q.inverse, s);                            \
      case PASS_ROW_GROUP:                                                                        \
        return q.fp64 ? row_group_launch<double, m>(q.row_descs, q.starts, q.ngroups, q.total, q.cb, q.nr, s) \
                      : row_group_launch<float, m>(q.row_descs, q.starts, q.ngroups, q.total, q.cb, q.nr, s); \
      case PASS_COL_GROUP:                                                                        \
        return q.fp64 ? col_group_launch<double, m>(q.nc, q.col_descs, q.starts, q.ngroups, q.total, s) \
                      : col_group_launch<float, m>(q.nc, q.col_descs, q.starts, q.ngroups, q.total, s); \
      default:                                                                                    \
        return (int)hipErrorInvalidValue;                                                         \
    }

}  // namespace tbs

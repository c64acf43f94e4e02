// Device FFT core for the Born-series passes (CDNA4 / gfx950).
//
// One transform of length M is held by TPT = M/E threads, E complex values per
// thread, in the "strided" register layout: register j of thread t holds
// element t + j*TPT.  That layout is the input of the first Stockham stage and
// the output of the last one, so a pass can load a zero-padded line straight
// from HBM into registers (elements >= M/2 are the registers j >= E/2), run
// the transform, apply a point-wise operation in registers, and start the
// next transform without any reordering.
//
// Stage s has radix R_s and L_s = prod_{i<s} R_i.  Butterfly b (M/R_s of them;
// thread t owns b = t + q*TPT, q < E/R_s) reads elements b + r*M/R_s,
// multiplies element r by w_{L_s R_s}^{r (b mod L_s)}, does a DFT of size R_s
// and writes output r to (b / L_s) L_s R_s + (b mod L_s) + r L_s (Stockham
// autosort, natural order out).  Between stages the data goes through LDS.
// Twiddles come from a per-length table built in FP64 on the host and rounded
// once to the working precision (no recurrences): stage s uses
// tw[off_s + (r-1) L_s + k], k < L_s, 1 <= r < R_s.  The inverse transform
// conjugates them.  Transforms are unnormalised in both directions.
#pragma once

#include <hip/hip_runtime.h>

namespace tbs {

template <typename T>
struct cx {
  T x, y;
};

// Loads and stores of global-memory arrays through address-space-1 pointers.
// A pass that takes its arguments from a descriptor table in memory (the
// grouped launches) holds generic pointers whose address space the compiler
// cannot prove and would access them with flat instructions; a flat access
// also counts against the LDS wait counter, so every exchange barrier of the
// transforms would wait for the HBM loads and stores still in flight.
template <typename T>
using gvec2 = T __attribute__((ext_vector_type(2)));
template <typename T>
__device__ __forceinline__ cx<T> gld(const void* base, int64_t i) {
  const gvec2<T> r = ((const __attribute__((address_space(1))) gvec2<T>*)(const gvec2<T>*)base)[i];
  return cx<T>{r.x, r.y};
}
template <typename T>
__device__ __forceinline__ void gst(void* base, int64_t i, cx<T> v) {
  ((__attribute__((address_space(1))) gvec2<T>*)(gvec2<T>*)base)[i] = gvec2<T>{v.x, v.y};
}
template <typename U>
__device__ __forceinline__ U gld1(const void* base, int64_t i) {
  return ((const __attribute__((address_space(1))) U*)(const U*)base)[i];
}
template <typename U>
__device__ __forceinline__ void gst1(void* base, int64_t i, U v) {
  ((__attribute__((address_space(1))) U*)(U*)base)[i] = v;
}

template <typename T>
__host__ __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename T>
__host__ __device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return {a.x * s, a.y * s}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> cconj(cx<T> a) { return {a.x, -a.y}; }

// Multiply by w4 = -i (forward) or +i (inverse).
template <bool INV, typename T>
__host__ __device__ __forceinline__ cx<T> rot4(cx<T> a) {
  if constexpr (INV) return {-a.y, a.x};
  else return {a.y, -a.x};
}

// Multiply by the constant e^{-+ 2 pi i m / 16} (forward: minus).
template <bool INV, int m, typename T>
__host__ __device__ __forceinline__ cx<T> rot16(cx<T> a) {
  constexpr int mm = ((m % 16) + 16) % 16;
  const T c1 = T(0.92387953251128675613);   // cos(pi/8)
  const T s1 = T(0.38268343236508977173);   // sin(pi/8)
  const T h = T(0.70710678118654752440);    // sqrt(1/2)
  // e^{-2 pi i mm/16} = cos(theta) - i sin(theta), theta = pi mm / 8
  T c, s;
  if constexpr (mm == 0) return a;
  else if constexpr (mm == 4) return rot4<INV>(a);
  else if constexpr (mm == 8) return {-a.x, -a.y};
  else if constexpr (mm == 12) return rot4<!INV>(a);
  else {
    if constexpr (mm == 1) { c = c1; s = s1; }
    else if constexpr (mm == 2) { c = h; s = h; }
    else if constexpr (mm == 3) { c = s1; s = c1; }
    else if constexpr (mm == 5) { c = -s1; s = c1; }
    else if constexpr (mm == 6) { c = -h; s = h; }
    else if constexpr (mm == 7) { c = -c1; s = s1; }
    else if constexpr (mm == 9) { c = -c1; s = -s1; }
    else if constexpr (mm == 10) { c = -h; s = -h; }
    else if constexpr (mm == 11) { c = -s1; s = -c1; }
    else if constexpr (mm == 13) { c = s1; s = -c1; }
    else if constexpr (mm == 14) { c = h; s = -h; }
    else { c = c1; s = -s1; }
    // forward multiplier (c - i s); inverse (c + i s)
    if constexpr (INV) return {a.x * c - a.y * s, a.x * s + a.y * c};
    else return {a.x * c + a.y * s, a.y * c - a.x * s};
  }
}

// ---- in-register DFTs, natural order in and out, on a[o + i*st] ----------

template <bool INV, typename T>
__host__ __device__ __forceinline__ void dft2(cx<T>& a, cx<T>& b) {
  const cx<T> t = a;
  a = t + b;
  b = t - b;
}

template <bool INV, typename T>
__host__ __device__ __forceinline__ void dft4(cx<T>& a0, cx<T>& a1, cx<T>& a2, cx<T>& a3) {
  const cx<T> t0 = a0 + a2, t1 = a0 - a2, t2 = a1 + a3, t3 = rot4<INV>(a1 - a3);
  a0 = t0 + t2;
  a2 = t0 - t2;
  a1 = t1 + t3;
  a3 = t1 - t3;
}

// DFT-3 (natural order): X0 = a+b+c, X1,2 = a - (b+c)/2 -+ i (sqrt3/2)(b-c)
template <bool INV, typename T>
__host__ __device__ __forceinline__ void dft3(cx<T>& a0, cx<T>& a1, cx<T>& a2) {
  const T s3 = T(0.86602540378443864676);
  const cx<T> s = a1 + a2, d = a1 - a2;
  const cx<T> m = {a0.x - T(0.5) * s.x, a0.y - T(0.5) * s.y};
  // forward: X1 = m - i s3 d, X2 = m + i s3 d
  const cx<T> id = INV ? cx<T>{-s3 * d.y, s3 * d.x} : cx<T>{s3 * d.y, -s3 * d.x};
  a0 = a0 + s;
  a1 = m + id;
  a2 = m - id;
}

// DFT-5 (natural order), Winograd-style with the real/imaginary constants of
// w5 = e^{-2 pi i/5}.
template <bool INV, typename T>
__host__ __device__ __forceinline__ void dft5(cx<T>& a0, cx<T>& a1, cx<T>& a2, cx<T>& a3, cx<T>& a4) {
  const T c1 = T(0.30901699437494742410);    // cos(2pi/5)
  const T c2 = T(-0.80901699437494742410);   // cos(4pi/5)
  const T s1 = T(0.95105651629515357212);    // sin(2pi/5)
  const T s2 = T(0.58778525229247312917);    // sin(4pi/5)
  const cx<T> b1 = a1 + a4, b4 = a1 - a4, b2 = a2 + a3, b3 = a2 - a3;
  const cx<T> m1 = {a0.x + c1 * b1.x + c2 * b2.x, a0.y + c1 * b1.y + c2 * b2.y};
  const cx<T> m2 = {a0.x + c2 * b1.x + c1 * b2.x, a0.y + c2 * b1.y + c1 * b2.y};
  // n1 = s1 b4 + s2 b3 ; n2 = s2 b4 - s1 b3
  const cx<T> n1 = {s1 * b4.x + s2 * b3.x, s1 * b4.y + s2 * b3.y};
  const cx<T> n2 = {s2 * b4.x - s1 * b3.x, s2 * b4.y - s1 * b3.y};
  // forward: X1 = m1 - i n1, X4 = m1 + i n1, X2 = m2 - i n2, X3 = m2 + i n2
  const cx<T> in1 = INV ? cx<T>{-n1.y, n1.x} : cx<T>{n1.y, -n1.x};
  const cx<T> in2 = INV ? cx<T>{-n2.y, n2.x} : cx<T>{n2.y, -n2.x};
  a0 = a0 + b1 + b2;
  a1 = m1 + in1;
  a4 = m1 - in1;
  a2 = m2 + in2;
  a3 = m2 - in2;
}

template <bool INV, typename T>
__host__ __device__ __forceinline__ void dft8(cx<T> (&a)[8]) {
  // radix-2 DIT split: X[k] = E[k] + w8^k O[k], X[k+4] = E[k] - w8^k O[k]
  cx<T> e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6];
  cx<T> o0 = a[1], o1 = a[3], o2 = a[5], o3 = a[7];
  dft4<INV>(e0, e1, e2, e3);
  dft4<INV>(o0, o1, o2, o3);
  o1 = rot16<INV, 2>(o1);
  o2 = rot16<INV, 4>(o2);
  o3 = rot16<INV, 6>(o3);
  a[0] = e0 + o0; a[4] = e0 - o0;
  a[1] = e1 + o1; a[5] = e1 - o1;
  a[2] = e2 + o2; a[6] = e2 - o2;
  a[3] = e3 + o3; a[7] = e3 - o3;
}

template <bool INV, typename T>
__host__ __device__ __forceinline__ void dft16(cx<T> (&a)[16]) {
  // 4 x 4: n = 4 n1 + n2, k = k1 + 4 k2
  cx<T> b[16];  // b[4*k1 + n2]
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    cx<T> x0 = a[n2], x1 = a[4 + n2], x2 = a[8 + n2], x3 = a[12 + n2];
    dft4<INV>(x0, x1, x2, x3);
    b[0 + n2] = x0;
    b[4 + n2] = x1;
    b[8 + n2] = x2;
    b[12 + n2] = x3;
  }
  // twiddles w16^{n2 k1}
  b[4 + 1] = rot16<INV, 1>(b[4 + 1]);
  b[4 + 2] = rot16<INV, 2>(b[4 + 2]);
  b[4 + 3] = rot16<INV, 3>(b[4 + 3]);
  b[8 + 1] = rot16<INV, 2>(b[8 + 1]);
  b[8 + 2] = rot16<INV, 4>(b[8 + 2]);
  b[8 + 3] = rot16<INV, 6>(b[8 + 3]);
  b[12 + 1] = rot16<INV, 3>(b[12 + 1]);
  b[12 + 2] = rot16<INV, 6>(b[12 + 2]);
  b[12 + 3] = rot16<INV, 9>(b[12 + 3]);
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    cx<T> x0 = b[4 * k1 + 0], x1 = b[4 * k1 + 1], x2 = b[4 * k1 + 2], x3 = b[4 * k1 + 3];
    dft4<INV>(x0, x1, x2, x3);
    a[k1 + 0] = x0;
    a[k1 + 4] = x1;
    a[k1 + 8] = x2;
    a[k1 + 12] = x3;
  }
}

template <int R, bool INV, typename T>
__host__ __device__ __forceinline__ void dft(cx<T> (&a)[R]) {
  if constexpr (R == 1) {
  } else if constexpr (R == 2) {
    dft2<INV>(a[0], a[1]);
  } else if constexpr (R == 3) {
    dft3<INV>(a[0], a[1], a[2]);
  } else if constexpr (R == 4) {
    dft4<INV>(a[0], a[1], a[2], a[3]);
  } else if constexpr (R == 5) {
    dft5<INV>(a[0], a[1], a[2], a[3], a[4]);
  } else if constexpr (R == 8) {
    dft8<INV>(a);
  } else if constexpr (R == 16) {
    dft16<INV>(a);
  } else {
    static_assert(R == 16, "unsupported radix");
  }
}

// ---- DFTs of R values whose upper half is zero ----------------------------
// The first stage of a transform of a zero-padded line (the upper half of
// the line is zero: registers j >= E/2, i.e. inputs r >= R/2 of every
// first-stage butterfly).  Under IEEE rules x + 0 is not x (for x = -0), so
// the compiler keeps those additions; these forms leave them out.  Outputs
// equal the full DFT's up to the sign of zero results.

// X_k = sum_{r < R/2} a_r w_R^{rk}, R = 4: X0,2 = a0 +- a1, X1,3 = a0 +- w4 a1.
template <bool INV, typename T>
__host__ __device__ __forceinline__ void dft4_half(cx<T>& a0, cx<T>& a1, cx<T>& a2, cx<T>& a3) {
  const cx<T> b = rot4<INV>(a1);
  a2 = a0 - a1;
  a3 = a0 - b;
  const cx<T> x0 = a0;
  a0 = x0 + a1;
  a1 = x0 + b;
}

template <int R, bool INV, typename T>
__host__ __device__ __forceinline__ void dft_half(cx<T> (&a)[R]) {
  if constexpr (R == 2) {
    a[1] = a[0];
  } else if constexpr (R == 4) {
    dft4_half<INV>(a[0], a[1], a[2], a[3]);
  } else if constexpr (R == 8) {
    // radix-2 DIT split: the even and the odd halves each have their upper
    // two inputs zero
    cx<T> e0 = a[0], e1 = a[2], e2, e3;
    cx<T> o0 = a[1], o1 = a[3], o2, o3;
    dft4_half<INV>(e0, e1, e2, e3);
    dft4_half<INV>(o0, o1, o2, o3);
    o1 = rot16<INV, 2>(o1);
    o2 = rot16<INV, 4>(o2);
    o3 = rot16<INV, 6>(o3);
    a[0] = e0 + o0; a[4] = e0 - o0;
    a[1] = e1 + o1; a[5] = e1 - o1;
    a[2] = e2 + o2; a[6] = e2 - o2;
    a[3] = e3 + o3; a[7] = e3 - o3;
  } else if constexpr (R == 16) {
    // 4 x 4 as in dft16: the first-level DFTs take a[n2], a[4+n2] (a[8+n2],
    // a[12+n2] are zero)
    cx<T> b[16];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
      cx<T> x0 = a[n2], x1 = a[4 + n2], x2, x3;
      dft4_half<INV>(x0, x1, x2, x3);
      b[0 + n2] = x0;
      b[4 + n2] = x1;
      b[8 + n2] = x2;
      b[12 + n2] = x3;
    }
    b[4 + 1] = rot16<INV, 1>(b[4 + 1]);
    b[4 + 2] = rot16<INV, 2>(b[4 + 2]);
    b[4 + 3] = rot16<INV, 3>(b[4 + 3]);
    b[8 + 1] = rot16<INV, 2>(b[8 + 1]);
    b[8 + 2] = rot16<INV, 4>(b[8 + 2]);
    b[8 + 3] = rot16<INV, 6>(b[8 + 3]);
    b[12 + 1] = rot16<INV, 3>(b[12 + 1]);
    b[12 + 2] = rot16<INV, 6>(b[12 + 2]);
    b[12 + 3] = rot16<INV, 9>(b[12 + 3]);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      cx<T> x0 = b[4 * k1 + 0], x1 = b[4 * k1 + 1], x2 = b[4 * k1 + 2], x3 = b[4 * k1 + 3];
      dft4<INV>(x0, x1, x2, x3);
      a[k1 + 0] = x0;
      a[k1 + 4] = x1;
      a[k1 + 8] = x2;
      a[k1 + 12] = x3;
    }
  } else {
    static_assert(R % 2 == 0, "a zero upper half needs an even radix");
  }
}

// ---- stage plan -----------------------------------------------------------

struct Stages {
  int n;
  int r[12];
};

// Radices for length M with E values per thread: each radix divides E; the
// largest admissible power of two first, then 3s and 5s.
__host__ __device__ constexpr Stages make_stages(int M, int E) {
  Stages s{0, {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0}};
  int rem = M;
  // powers of two
  while (rem % 2 == 0) {
    int r = 1;
    while (r * 2 <= E && E % (r * 2) == 0 && rem % (r * 2) == 0 && r * 2 <= 16) r *= 2;
    s.r[s.n++] = r;
    rem /= r;
  }
  while (rem % 5 == 0) {
    s.r[s.n++] = 5;
    rem /= 5;
  }
  while (rem % 3 == 0) {
    s.r[s.n++] = 3;
    rem /= 3;
  }
  if (rem != 1) s.n = -1;  // not 5-smooth
  return s;
}

__host__ __device__ constexpr bool stages_ok(int M, int E) {
  Stages s = make_stages(M, E);
  if (s.n <= 0 || M % E != 0) return false;
  for (int i = 0; i < s.n; ++i)
    if (E % s.r[i] != 0) return false;
  return true;
}

__host__ __device__ constexpr int stage_L(int M, int E, int S) {
  Stages s = make_stages(M, E);
  int L = 1;
  for (int i = 0; i < S; ++i) L *= s.r[i];
  return L;
}

__host__ __device__ constexpr int stage_twoff(int M, int E, int S) {
  Stages s = make_stages(M, E);
  int off = 0, L = 1;
  for (int i = 0; i < S; ++i) {
    off += (s.r[i] - 1) * L;
    L *= s.r[i];
  }
  return off;
}

// Index of output r of butterfly b in a stage of radix R and span L.
__host__ __device__ constexpr int stage_out_index(int b, int L, int R, int r) {
  return (b / L) * L * R + b % L + r * L;
}

// When L is a multiple of TPT (a stage after which every thread reads back
// exactly the values it wrote): the register j' that receives output r of the
// thread's butterfly q, i.e. (stage_out_index(t + q TPT, L, R, r) - t) / TPT.
__host__ __device__ constexpr int local_register(int q, int r, int TPT, int L, int R) {
  return (TPT * q / L) * (L * R / TPT) + (TPT * q) % L / TPT + r * (L / TPT);
}

__host__ __device__ constexpr bool stage_is_local(int M, int E, int S) {
  return S + 1 < make_stages(M, E).n && stage_L(M, E, S) % (M / E) == 0;
}

// ---- register-resident twiddles -------------------------------------------
// Butterfly q of stage S >= 1 in thread t twists its inputs by the factors of
// k = (t + q TPT) mod L.  k depends on q only through q TPT mod L, whose
// period is L / gcd(TPT, L), so a thread needs tw_classes(S) * (R - 1)
// factors per stage; a kernel that runs several transforms of one length
// (forward and inverse use the same factors, conjugated) loads them once.
__host__ __device__ constexpr int gcd_int(int a, int b) { return b == 0 ? a : gcd_int(b, a % b); }
__host__ __device__ constexpr int tw_classes(int M, int E, int S) {
  const int L = stage_L(M, E, S);
  const int NB = E / make_stages(M, E).r[S];
  const int P = L / gcd_int(M / E, L);
  return P < NB ? P : NB;
}
__host__ __device__ constexpr int tw_cache_base(int M, int E, int S) {
  int n = 0;
  for (int i = 1; i < S; ++i) n += tw_classes(M, E, i) * (make_stages(M, E).r[i] - 1);
  return n;
}
__host__ __device__ constexpr int tw_cache_size(int M, int E) {
  const int n = tw_cache_base(M, E, make_stages(M, E).n);
  return n > 0 ? n : 1;
}

// LDS index with one pad slot per 2^TBS_LDS_PAD_SHIFT elements (breaks
// power-of-two strides).
#ifndef TBS_LDS_PAD_SHIFT
#define TBS_LDS_PAD_SHIFT 4
#endif
__host__ __device__ constexpr int lpad(int i) { return i + (i >> TBS_LDS_PAD_SHIFT); }
// Slots per line of a block: the padded line plus a gap that moves the next
// line onto other banks (32 banks of 4 bytes, 16 lanes served per cycle for
// 8-byte accesses).  With 8-byte slots and two lines per block, half of each
// 16-lane group reads or writes the second line: a gap of 8 slots puts it on
// the other 16 banks.  Other shapes keep a gap of 4.
__host__ __device__ constexpr int lds_len(int M, int lines, int esz) {
  return M + (M >> TBS_LDS_PAD_SHIFT) + ((esz == 8 && lines == 2) ? 8 : 4);
}

// The same padded slots written so that the compiler sees one base address
// per thread plus constant offsets (the ds instructions' immediate field):
// (x + c) >> s == (x >> s) + (c >> s) whenever c is a multiple of 2^s.
//   read_slot : lpad(t + j TPT)
//   write_slot: lpad(stage_out_index(t + q TPT, L, R, r))
__host__ __device__ constexpr int read_slot(int TPT, int t, int j) {
  return (TPT % (1 << TBS_LDS_PAD_SHIFT) == 0) ? lpad(t) + j * lpad(TPT) : lpad(t + j * TPT);
}
__host__ __device__ constexpr int write_slot(int TPT, int L, int R, int t, int q, int r) {
  return (L % (1 << TBS_LDS_PAD_SHIFT) == 0 && (TPT * R) % (1 << TBS_LDS_PAD_SHIFT) == 0 && TPT % L == 0)
             ? lpad((t / L) * L * R + t % L) + q * lpad(TPT * R) + r * lpad(L)
         : (L == 1 && R == (1 << TBS_LDS_PAD_SHIFT))
             ? (t + q * TPT) * (R + 1) + r
             : lpad(stage_out_index(t + q * TPT, L, R, r));
}

// XOR layout of one exchange (the writes of a stage of radix R and span L and
// the reads of the next stage), used where L and R are powers of two.  LDS
// serves G = 128 / (bytes per element) lanes of one instruction per cycle (32
// banks of 4 bytes), conflict-free when their element indices differ mod G.
// The reads touch G consecutive indices: distinct mod G under any XOR of the
// low bits by a value taken from bits above them.  The writes touch G/L runs
// of L consecutive indices at stride L R (or, for L R < G, R windows of G
// indices that repeat the same residues): flipping bits [log2 L, log2 L + nb)
// by the run (window) number read from bits [s, s + nb) spreads them over
// all banks.  The padded layout above leaves 2- to 4-way conflicts on the
// radix-4 stages of 3 * 2^a and 5 * 2^a lines (L = 4) and on all stages with
// L < 16 of 8- and 16-byte elements where L R > 16.  Indices stay inside
// their aligned block of G (M a multiple of G), so the line needs M slots.
#ifndef TBS_LDS_SWIZZLE
#define TBS_LDS_SWIZZLE 1
#endif
struct Swz {
  int s, nb, tb;  // source bit, width, target bit; nb < 0: padded layout
};
__host__ __device__ constexpr bool pow2_int(int x) { return x > 0 && (x & (x - 1)) == 0; }
__host__ __device__ constexpr int log2_int(int x) {
  int n = 0;
  while ((1 << n) < x) ++n;
  return n;
}
// Whether the padded layout serves the writes of stage (L, R) and the reads
// of the next stage in the first wave without bank conflicts (butterfly 0
// and register 0: the others are the same patterns shifted by multiples of
// 16 elements).  Elements of 128 / G bytes cover 32 / G consecutive banks.
__host__ __device__ constexpr bool pad_group_ok(int a, int b, int words) {
  for (int d = 0; d < words; ++d)
    for (int e = 0; e < words; ++e)
      if ((a * words + d) % 32 == (b * words + e) % 32 && a != b) return false;
  return true;
}
__host__ __device__ constexpr bool pad_conflict_free(int TPT, int L, int R, int G) {
  const int words = 32 / G;
  const int lanes = TPT < 64 ? TPT : 64;
  for (int g0 = 0; g0 < lanes; g0 += G)
    for (int i = g0 + 1; i < g0 + G && i < lanes; ++i)
      for (int k = g0; k < i; ++k) {
        if (!pad_group_ok(read_slot(TPT, i, 0), read_slot(TPT, k, 0), words)) return false;
        for (int r = 0; r < R; ++r)
          if (!pad_group_ok(write_slot(TPT, L, R, i, 0, r), write_slot(TPT, L, R, k, 0, r), words))
            return false;
      }
  return true;
}
// The layout of one exchange: the padded one where it is conflict-free (its
// slots fold into the instructions' offsets), else the XOR layout.
__host__ __device__ constexpr Swz swz_of(int M, int TPT, int L, int R, int G) {
  if (!TBS_LDS_SWIZZLE || !pow2_int(L) || !pow2_int(R) || M % G != 0 ||
      pad_conflict_free(TPT, L, R, G))
    return Swz{0, -1, 0};
  if (L >= G) return Swz{0, 0, log2_int(L)};  // runs of G or more: plain indices
  return L * R >= G ? Swz{log2_int(L * R), log2_int(G / L), log2_int(L)}
                    : Swz{log2_int(G), log2_int(R), log2_int(L)};
}
__host__ __device__ constexpr int swz_apply(int e, Swz p) {
  return e ^ (((e >> p.s) & ((1 << p.nb) - 1)) << p.tb);
}
// Reads of the next stage: element t + j TPT.  With TPT a multiple of
// 2^(s + nb) the XOR mask does not depend on j (one base, constant offsets);
// with TPT a divisor of 2^s (t >> s == 0) and a multiple of 2^(tb + nb) it
// depends on j alone: 2^nb bases t ^ (c << tb), constant offsets.
__host__ __device__ constexpr int xread_slot(Swz p, int TPT, int t, int j) {
  return p.nb < 0 ? read_slot(TPT, t, j)
         : (TPT % (1 << (p.s + p.nb)) == 0) ? swz_apply(t, p) + j * TPT
         : ((1 << p.s) % TPT == 0 && TPT % (1 << (p.tb + p.nb)) == 0)
             ? (t ^ ((((j * TPT) >> p.s) & ((1 << p.nb) - 1)) << p.tb)) + j * TPT
             : swz_apply(t + j * TPT, p);
}
// Writes: output r of butterfly t + q TPT.  base = (t / L) L R + t mod L has
// zeros in bits [log2 L, log2 L R), and the mask bits come from above s >=
// log2 L R, so the slot is base + ((r ^ mask) << log2 L) + q TPT R when TPT
// is a multiple of L and TPT R one of 2^(s + nb).  Splitting r = rh 2^nb +
// rl, that is base + ((rl ^ mask) << tb) + (rh << (tb + nb)) + q TPT R:
// 2^nb bases per thread, the rest constant offsets.
__host__ __device__ constexpr bool xwrite_fast(Swz p, int TPT, int L, int R) {
  return p.nb >= 0 && TPT % L == 0 && (TPT * R) % (1 << (p.s + p.nb)) == 0;
}
__host__ __device__ constexpr int xwrite_base(Swz p, int L, int R, int t, int rl) {
  const int base = (t / L) * L * R + t % L;
  return base + ((rl ^ ((base >> p.s) & ((1 << p.nb) - 1))) << p.tb);
}
__host__ __device__ constexpr int xwrite_slot(Swz p, int TPT, int L, int R, int t, int q, int r) {
  if (p.nb < 0) return write_slot(TPT, L, R, t, q, r);
  if (xwrite_fast(p, TPT, L, R))
    return xwrite_base(p, L, R, t, r & ((1 << p.nb) - 1)) + ((r >> p.nb) << (p.tb + p.nb)) + q * TPT * R;
  return swz_apply(stage_out_index(t + q * TPT, L, R, r), p);
}

// One Stockham stage S and the exchange to stage S+1 (recursively).
// SPLIT: exchange real and imaginary parts in two rounds through a scalar LDS
// buffer of M (+pad) values, halving the LDS a line needs (four barriers per
// exchange instead of two).  Otherwise complex values go through LDS at once.
// TWC: the twiddle factors come from twc (tw_load), else from the table tw.
template <typename T, int M, int E, bool INV, bool SPLIT, bool TWC, int S, bool ZIN>
__device__ __forceinline__ void fft_stages(cx<T> (&v)[E], void* __restrict__ shv,
                                           const cx<T>* __restrict__ tw, const cx<T>* twc, int t) {
  constexpr Stages st = make_stages(M, E);
  static_assert(st.n > 0, "length not 5-smooth");
  constexpr int R = st.r[S];
  constexpr int L = stage_L(M, E, S);
  constexpr int TPT = M / E;
  constexpr int NB = E / R;
  constexpr int OFF = stage_twoff(M, E, S);
  constexpr int TWB = tw_cache_base(M, E, S);
  constexpr int TWN = tw_classes(M, E, S);
  constexpr bool LAST = (S + 1 == st.n);
  // Once L is a multiple of TPT, output r of butterfly b = t + q TPT lands on
  // index t + j' TPT with j' fixed by (q, r): the reader is the writing thread
  // itself, so the exchange is a register renaming (no LDS, no barrier).
  constexpr bool LOCAL = stage_is_local(M, E, S);
  constexpr Swz XL = swz_of(M, TPT, L, R, 128 / (SPLIT ? (int)sizeof(T) : 2 * (int)sizeof(T)));
  cx<T> w[LOCAL ? E : 1];
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int b = t + q * TPT;
    const int k = b % L;
    cx<T> a[R];
#pragma unroll
    for (int r = 0; r < R; ++r) a[r] = v[q + r * NB];
    if constexpr (S > 0) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const cx<T> w = TWC ? twc[TWB + (q % TWN) * (R - 1) + r - 1] : gld<T>(tw, OFF + (r - 1) * L + k);
        a[r] = INV ? cmulc(a[r], w) : cmul(a[r], w);
      }
    }
    // a zero-padded line (ZIN): the first stage's inputs r >= R/2 are the
    // zero upper half of the registers
    if constexpr (ZIN && S == 0 && R % 2 == 0 && (R / 2) * NB == E / 2) dft_half<R, INV>(a);
    else dft<R, INV>(a);
    if constexpr (LOCAL) {
#pragma unroll
      for (int r = 0; r < R; ++r)
        w[local_register(q, r, TPT, L, R)] = a[r];
    } else if constexpr (LAST || SPLIT) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[q + r * NB] = a[r];
    } else {
      cx<T>* sh = (cx<T>*)shv;
#pragma unroll
      for (int r = 0; r < R; ++r) sh[xwrite_slot(XL, TPT, L, R, t, q, r)] = a[r];
    }
  }
  if constexpr (LOCAL) {
#pragma unroll
    for (int j = 0; j < E; ++j) v[j] = w[j];
    fft_stages<T, M, E, INV, SPLIT, TWC, S + 1, ZIN>(v, shv, tw, twc, t);
  } else if constexpr (!LAST) {
    if constexpr (SPLIT) {
      T* sh = (T*)shv;
#pragma unroll
      for (int q = 0; q < NB; ++q) {
#pragma unroll
        for (int r = 0; r < R; ++r) sh[xwrite_slot(XL, TPT, L, R, t, q, r)] = v[q + r * NB].x;
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < E; ++j) v[j].x = sh[xread_slot(XL, TPT, t, j)];
      __syncthreads();
#pragma unroll
      for (int q = 0; q < NB; ++q) {
#pragma unroll
        for (int r = 0; r < R; ++r) sh[xwrite_slot(XL, TPT, L, R, t, q, r)] = v[q + r * NB].y;
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < E; ++j) v[j].y = sh[xread_slot(XL, TPT, t, j)];
      __syncthreads();
    } else {
      cx<T>* sh = (cx<T>*)shv;
      __syncthreads();
#pragma unroll
      for (int j = 0; j < E; ++j) v[j] = sh[xread_slot(XL, TPT, t, j)];
      __syncthreads();
    }
    fft_stages<T, M, E, INV, SPLIT, TWC, S + 1, ZIN>(v, shv, tw, twc, t);
  }
}

// Full transform of the thread's E registers (strided layout in and out).
// Every thread of the block must call it (it contains block barriers).
// shv: this line's LDS buffer, lds_len(M, .) elements of T (SPLIT) or cx<T>.
// ZIN: the registers j >= E/2 (the upper half of the line) hold zeros.
template <typename T, int M, int E, bool INV, bool SPLIT, bool ZIN = false>
__device__ __forceinline__ void fft(cx<T> (&v)[E], void* __restrict__ shv,
                                    const cx<T>* __restrict__ tw, int t) {
  fft_stages<T, M, E, INV, SPLIT, false, 0, ZIN>(v, shv, tw, nullptr, t);
}

// Loads the factors of stages S.. of thread t into twc (tw_cache_size(M, E)
// values), in the order fft_stages reads them.
template <typename T, int M, int E, int S = 1>
__device__ __forceinline__ void tw_load(cx<T>* twc, const cx<T>* __restrict__ tw, int t) {
  constexpr Stages st = make_stages(M, E);
  if constexpr (S < st.n) {
    constexpr int R = st.r[S];
    constexpr int L = stage_L(M, E, S);
    constexpr int OFF = stage_twoff(M, E, S);
    constexpr int NQ = tw_classes(M, E, S);
    constexpr int TWB = tw_cache_base(M, E, S);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int k = (t + q * (M / E)) % L;
#pragma unroll
      for (int r = 1; r < R; ++r) twc[TWB + q * (R - 1) + r - 1] = gld<T>(tw, OFF + (r - 1) * L + k);
    }
    tw_load<T, M, E, S + 1>(twc, tw, t);
  }
}

// The transform with the factors already in registers (tw_load).
template <typename T, int M, int E, bool INV, bool SPLIT, bool ZIN = false>
__device__ __forceinline__ void fft_cached(cx<T> (&v)[E], void* __restrict__ shv, const cx<T>* twc, int t) {
  fft_stages<T, M, E, INV, SPLIT, true, 0, ZIN>(v, shv, nullptr, twc, t);
}

}  // namespace tbs

// The paper's own periodic scheme on unpadded 2D grids (Sec. 2.2 Eq. of g~,
// Sec. 3.1, Algorithm 1): g~(p) = 1/(|p|^2 - k^2 - i eps) applied by FFTs of
// the grid's own (power-of-two) size, the fixed-point iteration
//   psi_{l+1} = ABL * (G(V psi_l) + psi0),   psi0 = G s,
// which by linearity equals the paper's ABL * ifft(g~ fft(V psi_l + S)) (and,
// with the k-space potential folded into the spectrum, its Case II form), and
// the centre-row relative L1 change as stopping error (Sec. 3.1 Eq. Error).
// The same passes run the convergent Born series the paper names as its
// extension: psi_1 = gamma psi0, psi_{l+1} = psi_l + gamma (G(V psi_l) + psi0
// - psi_l), gamma = i V / eps, computed from V in the row pass.
//
// Per iteration: one column pass (COL_CONV_FULL) and one row pass (k_iter_row)
// over the intermediate X[B][M/cb][rows][cb] of the padded solver, then a
// one-thread kernel that turns the check-row partial sums into the error and
// raises a device flag once it is below the tolerance; every later launch of
// the chunk sees the flag and returns at once, so the host only synchronises
// between chunks of iterations.
#include "tbs_passes.hpp"

namespace tbs {

template <typename T, int M, int E, int NR, int CB, bool SPLIT>
__global__ void __launch_bounds__(NR * (M / E)) TBS_OCCUPANCY(T, M, E, NR, SPLIT, 0)
    k_iter_row(IterArgs a) {
  if (a.done != nullptr && *a.done) return;
  constexpr int TPT = M / E;
  constexpr int NKB = M / CB;
  constexpr int LD = lds_len(M, NR, SPLIT ? sizeof(T) : 2 * sizeof(T));
  constexpr int NT = NR * TPT;
  constexpr int NW = (NT + 63) / 64;
  static_assert(TPT % CB == 0, "line too short for the column block");
  using LdsT = typename std::conditional<SPLIT, T, cx<T>>::type;
  __shared__ LdsT sh[NR * LD];
  __shared__ double red[2 * NW];

  const int lb = xcd_block(blockIdx.x, gridDim.x, 1);
  const int tid = threadIdx.x;
  const int tlo = tid % CB;
  const int r = (tid / CB) % NR;
  const int thi = tid / (CB * NR);
  const int t = thi * CB + tlo;
  const int rhs = lb % a.nrhs;
  const int rb = lb / a.nrhs;
  const int row = rb * NR + r;
  const bool valid = row < a.nrows;
  LdsT* shr = sh + r * LD;
  const cx<T>* tw = (const cx<T>*)a.tw;
  cx<T>* X = (cx<T>*)a.X;
  const int64_t P = (int64_t)a.nrows * a.nx;
  const int64_t srow = (int64_t)(valid ? row : 0) * a.nx;
  const int64_t sp_base = (int64_t)rhs * P + srow;
  const int64_t xbase = ((int64_t)rhs * NKB * a.nrows + (valid ? row : 0)) * CB;
  const int64_t kbstride = (int64_t)a.nrows * CB;
  cx<T>* psi = (cx<T>*)a.psi;
  cx<T>* psi0 = (cx<T>*)a.psi0;
  const cx<T>* Vp = (const cx<T>*)a.V;
  // the block holding the check row reduces its partial sums (block-uniform)
  const bool check_blk = a.mode == ITER_STEP && a.check_row >= rb * NR && a.check_row < rb * NR + NR;

  cx<T> v[E];
  double sd = 0.0, so = 0.0;
  if (a.mode == ITER_SOURCE) {
    const cx<T>* src = (const cx<T>*)a.src;
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int x = t + j * TPT;
      v[j] = (valid && x < a.nx) ? src[sp_base + x] : cx<T>{T(0), T(0)};
    }
  } else {
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int kx = t + j * TPT;
      v[j] = valid ? X[xbase + (int64_t)(kx / CB) * kbstride + (kx % CB)] : cx<T>{T(0), T(0)};
    }
    fft<T, M, E, true, SPLIT>(v, shr, tw, t);
    const double my = (a.mask_y != nullptr && valid) ? a.mask_y[row] : 1.0;
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int x = t + j * TPT;
      cx<T> w = {T(0), T(0)};
      if (valid && x < a.nx) {
        const int64_t i = sp_base + x;
        cx<T> f = v[j];
        cx<T> gam = {T(0), T(0)};
        if (a.cbs) {
          // gamma = i V / eps
          const cx<T> vv = Vp[srow + x];
          gam = cx<T>{(T)(-(double)vv.y * a.inv_eps), (T)((double)vv.x * a.inv_eps)};
        }
        if (a.mode == ITER_FIRST) {
          psi0[i] = f;
          if (a.cbs) f = cmul(gam, f);
        } else {
          const bool need_old = a.cbs || (check_blk && row == a.check_row);
          const cx<T> o = need_old ? psi[i] : cx<T>{T(0), T(0)};
          f = f + psi0[i];
          if (a.cbs) f = o + cmul(gam, f - o);
          if (a.mask_x != nullptr || a.mask_y != nullptr) {
            const T m = (T)(my * (a.mask_x != nullptr ? a.mask_x[x] : 1.0));
            f = cscale(f, m);
          }
          if (check_blk && row == a.check_row) {
            const double dr = (double)f.x - (double)o.x, di = (double)f.y - (double)o.y;
            sd += sqrt(dr * dr + di * di);
            so += sqrt((double)o.x * (double)o.x + (double)o.y * (double)o.y);
          }
        }
        psi[i] = f;
        w = Vp != nullptr ? cmul(f, Vp[srow + x]) : f;
      }
      v[j] = w;
    }
  }

  if (check_blk) {
    sd = wave_sum(sd);
    so = wave_sum(so);
    const int wv = tid >> 6;
    if ((tid & 63) == 0) {
      red[2 * wv] = sd;
      red[2 * wv + 1] = so;
    }
    __syncthreads();
    if (tid == 0) {
      double a0 = 0.0, a1 = 0.0;
      for (int k = 0; k < NW; ++k) {
        a0 += red[2 * k];
        a1 += red[2 * k + 1];
      }
      a.partials[2 * rhs] = a0;
      a.partials[2 * rhs + 1] = a1;
    }
  }

  fft<T, M, E, false, SPLIT>(v, shr, tw, t);
  if (valid) {
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int kx = t + j * TPT;
      X[xbase + (int64_t)(kx / CB) * kbstride + (kx % CB)] = v[j];
    }
  }
}

template <typename T, int M, int E, int NC, bool SPLIT>
__global__ void __launch_bounds__(NC * (M / E)) TBS_OCCUPANCY(T, M, E, NC, SPLIT, 0)
    k_iter_col(ColArgs a, const int* done) {
  if (done != nullptr && *done) return;
  col_pass_body<T, M, E, NC, COL_CONV_FULL, SPLIT>(a, xcd_block(blockIdx.x, gridDim.x, a.xcd_remap));
}

// Error of iteration `iter` (1-based): the largest over right-hand sides of
// sum |psi_new - psi_old| / sum |psi_old| on the check row; raises *done and
// records the count the first time it is below tol.  Skipped once done.
__global__ void k_iter_finish(const double* partials, int nrhs, int iter, double tol, double* errs,
                              int* done, int* iters) {
  if (threadIdx.x != 0 || *done) return;
  double e = 0.0;
  for (int b = 0; b < nrhs; ++b) {
    const double q = partials[2 * b] / partials[2 * b + 1];
    e = (q > e || q != q) ? q : e;
  }
  errs[iter - 1] = e;
  *iters = iter;
  if (e < tol) *done = 1;
}

// Folded periodic spectrum g~(p) / (Mx My) on [Mx/2+1][My/2+1] (the layout of
// the padded solver's table), and optionally g~(p) VV(p) / (Mx My) with the
// Case II k-space potential VV = eta |p|^(nu+1) - i (tau omega |p|^nu + eps)
// (Sec. 2.3.2 Eq. TBS_solution_absorbing-dispersive).  FP64, rounded once.
template <typename T>
__global__ void __launch_bounds__(256) k_periodic_green(cx<T>* ghat, cx<T>* ghat_vv, int64_t Mx,
                                                        int64_t My, double dx, double k2r,
                                                        double k2i, double eps, double tau,
                                                        double eta, double nu, double omega) {
  const int64_t hx = Mx / 2 + 1, hy = My / 2 + 1;
  const int64_t n = hx * hy;
  const double scale = 1.0 / ((double)Mx * (double)My);
  const double two_pi = 6.283185307179586476925286766559;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t ix = i / hy, iy = i % hy;
    const double px = two_pi * (double)ix / ((double)Mx * dx);
    const double py = two_pi * (double)iy / ((double)My * dx);
    const double p2 = px * px + py * py;
    // 1 / (a + i b) with a = p^2 - Re k^2, b = -(Im k^2 + eps)
    const double ar = p2 - k2r, bi = -(k2i + eps);
    const double den = ar * ar + bi * bi;
    const double gr = ar / den * scale, gi = -bi / den * scale;
    ghat[i] = cx<T>{(T)gr, (T)gi};
    if (ghat_vv != nullptr) {
      const double kmod = sqrt(p2);
      const double vr = eta * pow(kmod, nu + 1.0);
      const double vi = -(tau * omega * pow(kmod, nu) + eps);
      ghat_vv[i] = cx<T>{(T)(gr * vr - gi * vi), (T)(gr * vi + gi * vr)};
    }
  }
}

namespace {

template <typename T, int M>
int iter_row_launch(const IterArgs& a, hipStream_t s) {
  constexpr bool F64 = sizeof(T) == 8;
  constexpr int E = elems_per_thread(M, F64);
  // 4 rows per block where LDS allows (longer contiguous runs of the
  // intermediate per column block; measured faster on 4096^2)
  constexpr int NR = (M >= 2048 && row_fits(M, 4, (int)sizeof(cx<T>))) ? 4 : rows_per_block(M, F64);
  constexpr bool SP = split_lds(M, F64);
  const int grid = ((a.nrows + NR - 1) / NR) * a.nrhs;
  if (a.cb == 4) {
    hipLaunchKernelGGL((k_iter_row<T, M, E, NR, 4, SP>), dim3(grid), dim3(NR * (M / E)), 0, s, a);
  } else if (a.cb == 2) {
    hipLaunchKernelGGL((k_iter_row<T, M, E, NR, 2, SP>), dim3(grid), dim3(NR * (M / E)), 0, s, a);
  } else {
    return (int)hipErrorInvalidValue;
  }
  return (int)hipGetLastError();
}

template <typename T, int M>
int iter_col_launch(int nc, const ColArgs& a, const int* done, hipStream_t s) {
  constexpr bool F64 = sizeof(T) == 8;
  constexpr int E = elems_per_thread(M, F64);
  constexpr bool SP = split_lds(M, F64);
  constexpr int esz = (int)sizeof(cx<T>);
  const int grid = a.nrhs * a.n1 * a.n0;
  if constexpr (col_fits(M, 4, esz)) {
    if (nc == 4) {
      hipLaunchKernelGGL((k_iter_col<T, M, E, 4, SP>), dim3(grid), dim3(4 * (M / E)), 0, s, a, done);
      return (int)hipGetLastError();
    }
  }
  if constexpr (col_fits(M, 2, esz)) {
    if (nc == 2) {
      hipLaunchKernelGGL((k_iter_col<T, M, E, 2, SP>), dim3(grid), dim3(2 * (M / E)), 0, s, a, done);
      return (int)hipGetLastError();
    }
  }
  if (nc == 1) {
    hipLaunchKernelGGL((k_iter_col<T, M, E, 1, SP>), dim3(grid), dim3(M / E), 0, s, a, done);
    return (int)hipGetLastError();
  }
  return (int)hipErrorInvalidValue;
}

}  // namespace

#define TBS_ITER_ROW_CASE(m) \
  case m:                    \
    return fp64 ? iter_row_launch<double, m>(a, s) : iter_row_launch<float, m>(a, s);
#define TBS_ITER_COL_CASE(m) \
  case m:                    \
    return fp64 ? iter_col_launch<double, m>(nc, a, done, s) : iter_col_launch<float, m>(nc, a, done, s);

int launch_iter_row(bool fp64, int M, const IterArgs& a, hipStream_t s) {
  switch (M) {
    TBS_LENGTHS_POW2(TBS_ITER_ROW_CASE)
    default:
      return (int)hipErrorInvalidValue;
  }
}

int launch_iter_col(bool fp64, int M, int nc, const ColArgs& a, const int* done, hipStream_t s) {
  switch (M) {
    TBS_LENGTHS_POW2(TBS_ITER_COL_CASE)
    default:
      return (int)hipErrorInvalidValue;
  }
}

int launch_iter_finish(const double* partials, int nrhs, int iter, double tol, double* errs,
                       int* done, int* iters, hipStream_t s) {
  hipLaunchKernelGGL(k_iter_finish, dim3(1), dim3(64), 0, s, partials, nrhs, iter, tol, errs, done,
                     iters);
  return (int)hipGetLastError();
}

int launch_periodic_green(void* ghat, void* ghat_vv, bool fp64, int64_t Mx, int64_t My, double dx,
                          double k2r, double k2i, double eps, double tau, double eta, double nu,
                          double omega, hipStream_t s) {
  const int64_t n = (Mx / 2 + 1) * (My / 2 + 1);
  const int64_t blocks = (n + 255) / 256;
  const dim3 g((unsigned)(blocks < 65536 ? blocks : 65536));
  if (fp64)
    hipLaunchKernelGGL(k_periodic_green<double>, g, dim3(256), 0, s, (cx<double>*)ghat,
                       (cx<double>*)ghat_vv, Mx, My, dx, k2r, k2i, eps, tau, eta, nu, omega);
  else
    hipLaunchKernelGGL(k_periodic_green<float>, g, dim3(256), 0, s, (cx<float>*)ghat,
                       (cx<float>*)ghat_vv, Mx, My, dx, k2r, k2i, eps, tau, eta, nu, omega);
  return (int)hipGetLastError();
}

}  // namespace tbs

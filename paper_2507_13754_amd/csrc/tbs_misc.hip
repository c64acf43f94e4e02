// Elementwise and reduction kernels around the Born-series passes.
#include "tbs_fft.hpp"
#include "tbs_hankel.hpp"
#include "tbs_internal.hpp"

namespace tbs {

// residual[b][n] = sqrt(sum |u_n|^2) / sqrt(sum |p_{n+1}|^2), partials
// [n][b][nblk][2]; a fixed-order tree per (b, n), so the result is
// deterministic.  (Paper Sec. 3.1, Eq. Error, read as a whole-grid L2 norm.)
// Terms n >= nvalid are exactly zero (V = 0): residual 0.
__global__ void __launch_bounds__(256) k_finish_norms(const double* partials, int nterms, int nvalid,
                                                      int nrhs, int nblk, double* resid) {
  const int n = blockIdx.x % nterms;
  const int b = blockIdx.x / nterms;
  if (n >= nvalid) {
    if (threadIdx.x == 0) resid[(int64_t)b * nterms + n] = 0.0;
    return;
  }
  const double* pp = partials + 2 * ((int64_t)n * nrhs + b) * nblk;
  double su = 0.0, sp = 0.0;
  for (int k = threadIdx.x; k < nblk; k += 256) {
    su += pp[2 * k];
    sp += pp[2 * k + 1];
  }
  __shared__ double s0[256], s1[256];
  s0[threadIdx.x] = su;
  s1[threadIdx.x] = sp;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      s0[threadIdx.x] += s0[threadIdx.x + o];
      s1[threadIdx.x] += s1[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) resid[(int64_t)b * nterms + n] = sqrt(s0[0]) / sqrt(s1[0]);
}

int launch_finish_norms(const double* partials, int nterms, int nvalid, int nrhs, int nblk,
                        double* resid, hipStream_t s) {
  hipLaunchKernelGGL(k_finish_norms, dim3(nterms * nrhs), dim3(256), 0, s, partials, nterms, nvalid,
                     nrhs, nblk, resid);
  return (int)hipGetLastError();
}

// W on the padded periodic grid (paper Sec. 2.2, Eqs. soln_greens_fn and
// greens_fn): index i of an axis of size M holds the offset m = i (i <= M/2)
// or i - M; W(m) = dx^d g(k0, |m| dx) with g = (i/4) H0(k0 r) (2D) or
// e^{i k0 r}/(4 pi r) (3D); W(0) (the cell integral) is given.
__global__ void __launch_bounds__(256) k_green_eval(zd* W, int ndim, int64_t mx, int64_t my,
                                                    int64_t mz, double dx, zd k0, zd w0) {
  const int64_t n = mx * my * mz;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t ix = i % mx;
    const int64_t iy = (i / mx) % my;
    const int64_t iz = i / (mx * my);
    const double ox = (double)(ix <= mx / 2 ? ix : ix - mx);
    const double oy = (double)(iy <= my / 2 ? iy : iy - my);
    const double oz = (double)(iz <= mz / 2 ? iz : iz - mz);
    const double d2 = ox * ox + oy * oy + oz * oz;
    zd w;
    if (d2 == 0.0) {
      w = w0;
    } else {
      const double r = dx * sqrt(d2);
      const zd z = zscale(k0, r);
      if (ndim == 2) {
        zd h0, h1;
        hankel01(z, &h0, &h1);
        // dx^2 (i/4) H0
        w = zscale(zd{-h0.im, h0.re}, 0.25 * dx * dx);
      } else {
        const zd e = zexp(zd{-z.im, z.re});
        w = zscale(e, dx * dx * dx / (4.0 * kPi * r));
      }
    }
    W[i] = w;
  }
}

int launch_green_eval(void* W, int ndim, const int64_t* M, double dx, double k0r, double k0i,
                      double w0r, double w0i, hipStream_t s) {
  const int64_t n = M[0] * M[1] * M[2];
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_green_eval, dim3((unsigned)(blocks < 65536 * 8 ? blocks : 65536 * 8)),
                     dim3(256), 0, s, (zd*)W, ndim, M[0], M[1], M[2], dx, zd{k0r, k0i},
                     zd{w0r, w0i});
  return (int)hipGetLastError();
}

// Folded spectrum: ghat[fx][fy][fz] = What[fz][fy][fx] / (Mx My Mz) for
// f* in [0, M*/2]; exact because W_pad is even in every axis.
template <typename T>
__global__ void __launch_bounds__(256) k_green_fold(const zd* What, cx<T>* ghat, int64_t mx,
                                                    int64_t my, int64_t mz) {
  const int64_t hx = mx / 2 + 1, hy = my / 2 + 1, hz = mz / 2 + 1;
  const int64_t n = hx * hy * hz;
  const double sc = 1.0 / ((double)mx * (double)my * (double)mz);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t fz = i % hz;
    const int64_t fy = (i / hz) % hy;
    const int64_t fx = i / (hz * hy);
    const zd w = What[(fz * my + fy) * mx + fx];
    ghat[i] = cx<T>{(T)(w.re * sc), (T)(w.im * sc)};
  }
}

int launch_green_fold(const void* What, void* ghat, bool fp64, int ndim, const int64_t* M,
                      hipStream_t s) {
  (void)ndim;
  const int64_t n = (M[0] / 2 + 1) * (M[1] / 2 + 1) * (M[2] / 2 + 1);
  const int64_t blocks = (n + 255) / 256;
  const dim3 g((unsigned)(blocks < 65536 * 8 ? blocks : 65536 * 8));
  if (fp64)
    hipLaunchKernelGGL(k_green_fold<double>, g, dim3(256), 0, s, (const zd*)What,
                       (cx<double>*)ghat, M[0], M[1], M[2]);
  else
    hipLaunchKernelGGL(k_green_fold<float>, g, dim3(256), 0, s, (const zd*)What,
                       (cx<float>*)ghat, M[0], M[1], M[2]);
  return (int)hipGetLastError();
}

// V = k(c)^2 - k0^2 with k(c) = omega/c + a (disp + i)  (a = alpha0 omega^y,
// disp = tan(pi y/2), or 0 when y = 1), and dV/dc = -2 k omega / c^2.
// (Paper Sec. 2.1.2 and Sec. 2.3.3, Eq. TBS_equation_inhomogeneous.)
template <typename T>
__global__ void __launch_bounds__(256) k_potential(const double* c, cx<T>* V, cx<T>* dVdc,
                                                   int64_t n, double omega, double a_abs,
                                                   double disp, double k0sq_r, double k0sq_i) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double ci = c[i];
    const double kr = omega / ci + a_abs * disp;
    const double ki = a_abs;
    if (V) V[i] = cx<T>{(T)(kr * kr - ki * ki - k0sq_r), (T)(2.0 * kr * ki - k0sq_i)};
    if (dVdc) {
      const double f = -2.0 * omega / (ci * ci);
      dVdc[i] = cx<T>{(T)(f * kr), (T)(f * ki)};
    }
  }
}

int launch_potential(const double* c, void* V, void* dVdc, bool fp64, int64_t n, double omega,
                     double a_abs, double disp, double k0sq_r, double k0sq_i, hipStream_t s) {
  const int64_t blocks = (n + 255) / 256;
  const dim3 g((unsigned)(blocks < 65536 * 8 ? blocks : 65536 * 8));
  if (fp64)
    hipLaunchKernelGGL(k_potential<double>, g, dim3(256), 0, s, c, (cx<double>*)V,
                       (cx<double>*)dVdc, n, omega, a_abs, disp, k0sq_r, k0sq_i);
  else
    hipLaunchKernelGGL(k_potential<float>, g, dim3(256), 0, s, c, (cx<float>*)V,
                       (cx<float>*)dVdc, n, omega, a_abs, disp, k0sq_r, k0sq_i);
  return (int)hipGetLastError();
}

// S2 = coef * p1^2 / c^4 with coef = -(1/2)(1 + B/2A)(2 omega)^2 / rho
// (paper Sec. 2.3.4, Eq. TBS_solution_shi_2, local sound speed c).
template <typename T>
__global__ void __launch_bounds__(256) k_harmonic(const cx<T>* p1, const double* c, cx<T>* S2,
                                                  int64_t n, int nrhs, double coef) {
  const int64_t tot = n * nrhs;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tot;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double ci = c[i % n];
    const double f = coef / (ci * ci * ci * ci);
    const double pr = p1[i].x, pi = p1[i].y;
    S2[i] = cx<T>{(T)(f * (pr * pr - pi * pi)), (T)(f * 2.0 * pr * pi)};
  }
}

int launch_harmonic_source(const void* p1, const double* c, void* S2, bool fp64, int64_t n,
                           int nrhs, double coef, hipStream_t s) {
  const int64_t blocks = (n * nrhs + 255) / 256;
  const dim3 g((unsigned)(blocks < 65536 * 8 ? blocks : 65536 * 8));
  if (fp64)
    hipLaunchKernelGGL(k_harmonic<double>, g, dim3(256), 0, s, (const cx<double>*)p1, c,
                       (cx<double>*)S2, n, nrhs, coef);
  else
    hipLaunchKernelGGL(k_harmonic<float>, g, dim3(256), 0, s, (const cx<float>*)p1, c,
                       (cx<float>*)S2, n, nrhs, coef);
  return (int)hipGetLastError();
}

// n-th harmonic source from the lower harmonics (Sec. 2.3.4, Eqs. of the
// nonlinear solutions with sum terms): S_n = coef / c^4 * sum_{a=1}^{n-1}
// psi_a psi_{n-a} (ordered pairs, so the a = n-a term enters once), with
// coef = -(1/2)(1 + B/2A)(n omega)^2 / rho; products and sum in FP64.
// Scaled form: field a holds psi_a 2^{e_a} (unscale[a-1] = 2^{-e_a}) and the
// output is S_n 2^{e_n} (out_scale = 2^{e_n}); all of it in FP64, so fields
// far below the FP32 range keep their precision.
struct HarmonicFields {
  const void* f[TBS_HARMONIC_MAX - 1];
  double unscale[TBS_HARMONIC_MAX - 1];
};

template <typename T>
__device__ __forceinline__ void harmonic_value(const HarmonicFields& h, int n, const double* c, int64_t np,
                                               int64_t i, double coef, double& re, double& im) {
  double ar = 0.0, ai = 0.0;
  for (int a = 1; a <= n / 2; ++a) {
    const cx<T> x = ((const cx<T>*)h.f[a - 1])[i];
    const cx<T> y = ((const cx<T>*)h.f[n - a - 1])[i];
    const double w = ((2 * a == n) ? 1.0 : 2.0) * h.unscale[a - 1] * h.unscale[n - a - 1];
    ar += w * ((double)x.x * (double)y.x - (double)x.y * (double)y.y);
    ai += w * ((double)x.x * (double)y.y + (double)x.y * (double)y.x);
  }
  const double ci = c[i % np];
  const double g = coef / (ci * ci * ci * ci);
  re = g * ar;
  im = g * ai;
}

template <typename T>
__global__ void __launch_bounds__(256) k_harmonic_n(HarmonicFields h, int n, const double* c,
                                                    cx<T>* S, int64_t np, int nrhs, double coef,
                                                    double out_scale) {
  const int64_t tot = np * nrhs;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tot;
       i += (int64_t)gridDim.x * blockDim.x) {
    double re, im;
    harmonic_value<T>(h, n, c, np, i, coef, re, im);
    S[i] = cx<T>{(T)(re * out_scale), (T)(im * out_scale)};
  }
}

// Largest |S_n| (FP64, unscaled fields as above) per block of a fixed grid
// (kHarmMaxBlocks blocks), then over the blocks: partial[kHarmMaxBlocks] holds
// the result.  No atomics: the second kernel is one block.
constexpr int kHarmMaxBlocks = 1024;

template <typename T>
__global__ void __launch_bounds__(256) k_harmonic_n_max(HarmonicFields h, int n, const double* c,
                                                        int64_t np, int nrhs, double coef, double* partial) {
  __shared__ double red[256];
  const int64_t tot = np * nrhs;
  double m = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tot;
       i += (int64_t)gridDim.x * blockDim.x) {
    double re, im;
    harmonic_value<T>(h, n, c, np, i, coef, re, im);
    m = fmax(m, fmax(fabs(re), fabs(im)));
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) k_max_blocks(double* partial, int nb) {
  __shared__ double red[256];
  double m = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) m = fmax(m, partial[i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[nb] = red[0];
}

int launch_harmonic_source_n(int n, const void* const* fields, const double* unscale, const double* c,
                             void* S, bool fp64, int64_t np, int nrhs, double coef, double out_scale,
                             hipStream_t s) {
  HarmonicFields h{};
  for (int a = 0; a < n - 1; ++a) {
    h.f[a] = fields[a];
    h.unscale[a] = unscale ? unscale[a] : 1.0;
  }
  const int64_t blocks = (np * nrhs + 255) / 256;
  const dim3 g((unsigned)(blocks < 65536 * 8 ? blocks : 65536 * 8));
  if (fp64)
    hipLaunchKernelGGL(k_harmonic_n<double>, g, dim3(256), 0, s, h, n, c, (cx<double>*)S, np, nrhs,
                       coef, out_scale);
  else
    hipLaunchKernelGGL(k_harmonic_n<float>, g, dim3(256), 0, s, h, n, c, (cx<float>*)S, np, nrhs,
                       coef, out_scale);
  return (int)hipGetLastError();
}

int launch_harmonic_source_n_max(int n, const void* const* fields, const double* unscale, const double* c,
                                 bool fp64, int64_t np, int nrhs, double coef, double* partial,
                                 hipStream_t s) {
  HarmonicFields h{};
  for (int a = 0; a < n - 1; ++a) {
    h.f[a] = fields[a];
    h.unscale[a] = unscale ? unscale[a] : 1.0;
  }
  if (fp64)
    hipLaunchKernelGGL(k_harmonic_n_max<double>, dim3(kHarmMaxBlocks), dim3(256), 0, s, h, n, c, np, nrhs,
                       coef, partial);
  else
    hipLaunchKernelGGL(k_harmonic_n_max<float>, dim3(kHarmMaxBlocks), dim3(256), 0, s, h, n, c, np, nrhs,
                       coef, partial);
  hipLaunchKernelGGL(k_max_blocks, dim3(1), dim3(256), 0, s, partial, kHarmMaxBlocks);
  return (int)hipGetLastError();
}

// Receiver misfit: r = p[b][rec] - p_obs[b][r]; q[b][rec] += r (q zeroed by
// the caller; R^H sums receivers that share a cell); jpart[b][r] = |r|^2.
template <typename T>
__global__ void __launch_bounds__(256) k_misfit(const cx<T>* p, const int64_t* rec,
                                                const cx<T>* pobs, cx<T>* q, double* jpart,
                                                int64_t P, int nrec, int nrhs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrec * nrhs) return;
  const int b = i / nrec;
  const int r = i % nrec;
  const int64_t ri = rec[r];
  if (ri < 0 || ri >= P) {  // out-of-grid receiver: ignored
    jpart[i] = 0.0;
    return;
  }
  const int64_t idx = (int64_t)b * P + ri;
  const cx<T> d = p[idx] - pobs[i];
  atomicAdd(&q[idx].x, d.x);
  atomicAdd(&q[idx].y, d.y);
  jpart[i] = (double)d.x * d.x + (double)d.y * d.y;
}

int launch_misfit(const void* p, const int64_t* rec, const void* p_obs, void* q, double* jpart,
                  bool fp64, int64_t P, int nrec, int nrhs, hipStream_t s) {
  const int n = nrec * nrhs;
  if (fp64)
    hipLaunchKernelGGL(k_misfit<double>, dim3((n + 255) / 256), dim3(256), 0, s,
                       (const cx<double>*)p, rec, (const cx<double>*)p_obs, (cx<double>*)q, jpart,
                       P, nrec, nrhs);
  else
    hipLaunchKernelGGL(k_misfit<float>, dim3((n + 255) / 256), dim3(256), 0, s,
                       (const cx<float>*)p, rec, (const cx<float>*)p_obs, (cx<float>*)q, jpart, P,
                       nrec, nrhs);
  return (int)hipGetLastError();
}

// grad_c (+)= Re( sum_b g[b] * dV/dc )
template <typename T>
__global__ void __launch_bounds__(256) k_grad(const cx<T>* g, int nrhs, const cx<T>* dVdc,
                                              double* grad, int64_t P, int accumulate) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < P;
       i += (int64_t)gridDim.x * blockDim.x) {
    double sr = 0.0, si = 0.0;
    for (int b = 0; b < nrhs; ++b) {
      sr += g[(int64_t)b * P + i].x;
      si += g[(int64_t)b * P + i].y;
    }
    const double v = sr * (double)dVdc[i].x - si * (double)dVdc[i].y;
    grad[i] = accumulate ? grad[i] + v : v;
  }
}

int launch_grad_assemble(const void* g, int nrhs, const void* dVdc, double* grad_c, bool fp64,
                         int64_t P, int accumulate, hipStream_t s) {
  const int64_t blocks = (P + 255) / 256;
  const dim3 gr((unsigned)(blocks < 65536 * 8 ? blocks : 65536 * 8));
  if (fp64)
    hipLaunchKernelGGL(k_grad<double>, gr, dim3(256), 0, s, (const cx<double>*)g, nrhs,
                       (const cx<double>*)dVdc, grad_c, P, accumulate);
  else
    hipLaunchKernelGGL(k_grad<float>, gr, dim3(256), 0, s, (const cx<float>*)g, nrhs,
                       (const cx<float>*)dVdc, grad_c, P, accumulate);
  return (int)hipGetLastError();
}

// out[0] = 0.5 * sum(parts[0:n]) in a fixed order (one block).
__global__ void __launch_bounds__(256) k_sum_half(const double* parts, int n, double* out) {
  __shared__ double s[256];
  double a = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) a += parts[i];
  s[threadIdx.x] = a;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = 0.5 * s[0];
}

int launch_sum_half(const double* parts, int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_half, dim3(1), dim3(256), 0, s, parts, n, out);
  return (int)hipGetLastError();
}

// Fill with zeros through vector stores (graph-capture safe).
__global__ void __launch_bounds__(256) k_zero(uint2* p, int64_t n8) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n8;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = uint2{0u, 0u};
}

int launch_zero(void* p, int64_t bytes, hipStream_t s) {
  if (bytes % 8 != 0) return (int)hipErrorInvalidValue;
  const int64_t n8 = bytes / 8;
  if (n8 == 0) return 0;
  const int64_t blocks = (n8 + 255) / 256;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)(blocks < 65536 * 4 ? blocks : 65536 * 4)), dim3(256),
                     0, s, (uint2*)p, n8);
  return (int)hipGetLastError();
}

}  // namespace tbs

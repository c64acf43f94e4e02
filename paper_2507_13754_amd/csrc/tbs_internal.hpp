// Internal interfaces between the host runtime and the device passes.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace tbs {

// Row pass: one FFT line per grid row (x axis).  Spectral layout of the
// intermediate X: [rhs][M/CB][nrows][CB], CB = kBlock columns per block, rows
// ordered rho = y*nz + z (3D) / rho = y (2D).  Spatial arrays (source, p, c,
// V, pairing, gradient) are [rhs][z][y][x] / [z][y][x].
// ROW_IN_SOURCE: w = src; ROW_IN_SPECTRAL: u = crop(IFFT(X)); ROW_IN_SPATIAL:
// w = V src (restart of a series from a stored spatial term).
enum RowIn { ROW_IN_SOURCE = 0, ROW_IN_SPECTRAL = 1, ROW_IN_SPATIAL = 2 };
enum RowAcc { ACC_NONE = 0, ACC_INIT = 1, ACC_ADD = 2, ACC_PAIR = 3 };

// Spectral columns per contiguous block (cb) is 4, or 2 for FP64 plans with
// 4096+ long columns (see spectral_block).

struct RowArgs {
  void* X;              // spectral intermediate (in and/or out)
  const void* src;      // ROW_IN_SOURCE: source [rhs][P]
  const void* V;        // potential [P] (OUT) ; nullptr = multiply by 0
  void* p;              // accumulator [rhs][P]
  void* pstore;         // optional copy of the updated accumulator [rhs][P]
  void* ustore;         // optional copy of the term u itself [rhs][P]
  void* c;              // Kahan compensation [rhs][P], bf16 (re, im) pairs in 32 bits (FP32 only)
  const void* pair;     // ACC_PAIR: partial sums P_{L-1-m} [rhs][P]
  void* grad;           // ACC_PAIR: g_V accumulator [rhs][P]
  double* partials;     // [rhs][nblk] x 2 (|u|^2, |p|^2) for this term
  const void* tw;       // twiddles for M
  int nx, ny, nz;       // physical grid (nz = 1 in 2D)
  int nrows;            // ny * nz
  int nrhs;
  int in_mode, acc, out_spec, conj_v;
  int cb;
  int xcd_remap;
  // ROW_IN_SPATIAL (2D): subtract the density term div(gamma grad src) when
  // gamma (float64 [ny][nx]) is set; inv_dx2 = 1 / dx^2
  const double* gamma;
  double inv_dx2;
};

struct ColArgs {
  const void* in;
  void* out;
  const void* tw;
  const void* ghat;     // CONV: folded spectrum
  int op;               // COL_CONV / COL_FWD / COL_INV / COL_FULL
  int conj_g;
  int n_in, n_out;      // valid input length (zero above), stored outputs
  int64_t in_astride, out_astride;
  int64_t in_rs, in_s1, in_s0, out_rs, out_s1, out_s0;
  int nrhs, n1, n0;
  int cb;               // spectral block width of the layout
  int sub;              // blocks per layout block (block holds cb/sub columns); 1 otherwise
  int mirror;           // launch mirror-image columns (shared spectrum lines) back to back
  int zcols, zlim;      // column validity: i0*zcols + col/cb < zlim
  int mx, mm;           // fold sizes of kx (= i1*cb + col%cb) and kmid (= i0)
  int64_t g_sx, g_sm;   // table strides for fold(kx), fold(kmid)
  int xcd_remap;
};
// COL_CONV_FULL: the convolution on unpadded (periodic) lines, every value
// loaded and stored.
enum ColOp { COL_CONV = 0, COL_FWD = 1, COL_INV = 2, COL_FULL = 3, COL_CONV_FULL = 4 };

// Row pass of the paper's periodic fixed-point iteration on unpadded 2D grids
// (lines of M = N values, same intermediate layout as RowArgs).
enum IterMode {
  ITER_SOURCE = 0,  // w = s                       -> forward FFT -> X
  ITER_FIRST = 1,   // psi0 = IFFT(X); psi = psi0 (CBS: gamma psi0) -> w = V psi -> FFT -> X
  ITER_STEP = 2     // psi = mask (IFFT(X) + psi0) (CBS: mask (psi + gamma (IFFT(X) + psi0 - psi)))
                    //   -> w = V psi -> forward FFT -> X
};
struct IterArgs {
  void* X;
  const void* tw;
  void* psi;            // [B][ny][nx] current field (read at the check row, then overwritten)
  void* psi0;           // [B][ny][nx] G s
  const void* src;      // ITER_SOURCE: [B][ny][nx]
  const void* V;        // [ny][nx] or NULL (V = 1: the k-space potential lives in the spectrum)
  const double* mask_x; // [nx] or NULL
  const double* mask_y; // [ny] or NULL
  double* partials;     // ITER_STEP: [B][2] = sum |psi_new - psi_old|, sum |psi_old| on the check row
  const int* done;      // skip the launch when *done != 0 (NULL: never)
  int nx, nrows, nrhs;
  int mode;
  int check_row;
  int cb;
  int cbs;              // convergent Born series update (gamma = i V / eps), else the paper's
  double inv_eps;       // 1 / eps for gamma
};

// FFT lengths with compiled kernels: powers of two, 3 * 2^a and 5 * 2^a.
#define TBS_LENGTHS_POW2(X) X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096)
#define TBS_LENGTHS_THREE(X) X(48) X(96) X(192) X(384) X(768) X(1536) X(3072)
#define TBS_LENGTHS_FIVE(X) X(80) X(160) X(320) X(640) X(1280) X(2560)

enum PassKind { PASS_ROW = 0, PASS_COL = 1, PASS_ROW_FULL = 2, PASS_ROW_GROUP = 3, PASS_COL_GROUP = 4 };

// One launch request for the length-family dispatchers.
struct PassReq {
  int kind = PASS_ROW;
  bool fp64 = false;
  int M = 0;
  int nc = 0;                       // columns per block (column passes)
  int nr = 0;                       // rows per row-pass block (0: default)
  int cb = 4;                       // layout block width (grouped row passes)
  const RowArgs* row = nullptr;     // PASS_ROW
  int nblk_rows = 0;
  const ColArgs* col = nullptr;     // PASS_COL
  void* data = nullptr;             // PASS_ROW_FULL
  const void* tw = nullptr;
  int nrows = 0, inverse = 0;
  const RowArgs* row_descs = nullptr;  // grouped: device arrays
  const ColArgs* col_descs = nullptr;
  const int* starts = nullptr;
  int ngroups = 0, total = 0;
};
int dispatch_pow2(const PassReq& q, hipStream_t s);
int dispatch_three(const PassReq& q, hipStream_t s);
int dispatch_five(const PassReq& q, hipStream_t s);

// Lengths the library has kernels for.
bool fft_length_supported(int M);
int fft_supported_lengths(int* out, int cap);   // ascending
int fft_elems_per_thread(int M, bool fp64);
int row_rows_per_block(int M, bool fp64);
int spectral_block(int My, bool fp64);
int col_max_cols(int M, bool fp64);  // widest column block that fits LDS
int conv_cols_per_block(int M, bool fp64, int cb);  // columns per convolution block
// Launchers (return hipError_t as int).
int launch_row_pass(bool fp64, int M, const RowArgs& a, int nblk_rows, int nr, hipStream_t s);
// Block-shape candidates the autotuner may pick for a line length.
int row_nr_candidates(int M, bool fp64, int* out);      // returns count
int conv_nc_candidates(int M, bool fp64, int cb, int* out);
int launch_col_pass(bool fp64, int M, int NC, const ColArgs& a, hipStream_t s);
int launch_row_fft_full(int M, void* data, const void* tw, int nrows, int inverse, hipStream_t s);
// Grouped launches (descs/starts are device arrays of ngroups entries).
int launch_row_group(bool fp64, int M, int cb, int nr, const RowArgs* descs, const int* starts,
                     int ngroups, int total_blocks, hipStream_t s);
int launch_col_group(bool fp64, int M, int nc, const ColArgs* descs, const int* starts, int ngroups,
                     int total_blocks, hipStream_t s);

// Periodic (unpadded, power-of-two) passes of the paper's fixed-point iteration.
int launch_iter_row(bool fp64, int M, const IterArgs& a, hipStream_t s);
int launch_iter_col(bool fp64, int M, int nc, const ColArgs& a, const int* done, hipStream_t s);
int launch_iter_finish(const double* partials, int nrhs, int iter, double tol, double* errs,
                       int* done, int* iters, hipStream_t s);
int launch_periodic_green(void* ghat, void* ghat_vv, bool fp64, int64_t Mx, int64_t My, double dx,
                          double k2r, double k2i, double eps, double tau, double eta, double nu,
                          double omega, hipStream_t s);

// Elementwise / reduction kernels.
int launch_finish_norms(const double* partials, int nterms, int nvalid, int nrhs, int nblk,
                        double* resid, hipStream_t s);
int launch_green_eval(void* W, int ndim, const int64_t* M, double dx, double k0r, double k0i,
                      double w0r, double w0i, hipStream_t s);
int launch_green_fold(const void* What, void* ghat, bool fp64, int ndim, const int64_t* M,
                      hipStream_t s);
int launch_potential(const double* c, void* V, void* dVdc, bool fp64, int64_t n, double omega,
                     double a_abs, double disp, double k0sq_r, double k0sq_i, hipStream_t s);
int launch_harmonic_source(const void* p1, const double* c, void* S2, bool fp64, int64_t n,
                           int nrhs, double coef, hipStream_t s);
// highest harmonic order accepted by launch_harmonic_source_n
#define TBS_HARMONIC_MAX 9
// unscale: NULL or host double [n-1] (field a holds psi_a / unscale[a-1]);
// the output is multiplied by out_scale
int launch_harmonic_source_n(int n, const void* const* fields, const double* unscale, const double* c,
                             void* S, bool fp64, int64_t np, int nrhs, double coef, double out_scale,
                             hipStream_t s);
// max |Re|, |Im| of the unscaled S_n into partial[1024] (partial: dev double
// [1025]; partial[0..1023] are block maxima)
int launch_harmonic_source_n_max(int n, const void* const* fields, const double* unscale, const double* c,
                                 bool fp64, int64_t np, int nrhs, double coef, double* partial,
                                 hipStream_t s);
constexpr int kHarmonicMaxSlots = 1025;
int launch_misfit(const void* p, const int64_t* rec, const void* p_obs, void* q, double* jpart,
                  bool fp64, int64_t P, int nrec, int nrhs, hipStream_t s);
int launch_grad_assemble(const void* g, int nrhs, const void* dVdc, double* grad_c, bool fp64,
                         int64_t P, int accumulate, hipStream_t s);
int launch_zero(void* p, int64_t bytes, hipStream_t s);
int launch_sum_half(const double* parts, int n, double* out, hipStream_t s);

}  // namespace tbs

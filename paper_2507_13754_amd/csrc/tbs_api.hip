// Host runtime of the C ABI declared in include/tbs.h: plan validation and
// sizing, device buffers, FP64 twiddle tables, the Green tabulation
// sequence, and the per-term pass sequence of the Born series.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <map>
#include <mutex>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/tbs.h"
#include "tbs_fft.hpp"
#include "tbs_hankel.hpp"
#include "tbs_internal.hpp"

using tbs::zd;

#ifndef TBS_BATCH_CHAINS_DEFAULT
#define TBS_BATCH_CHAINS_DEFAULT 3
#endif
constexpr int kMaxChains = 4;
#ifndef TBS_BATCH_TILE_RHS_DEFAULT
#define TBS_BATCH_TILE_RHS_DEFAULT 2
#endif

struct tbs_plan {
  int ndim = 2;
  int64_t N[3] = {1, 1, 1};  // x, y, z
  int64_t M[3] = {1, 1, 1};
  double dx = 0.0;
  zd k0{0.0, 0.0};
  int dtype = TBS_C64;
  bool fp64 = false;
  int batch = 1;
  int cb = 4;
  int row_nr = 0;           // rows per row-pass block (autotuned; 0 = default)
  int conv_nc = 0;          // columns per convolution block (autotuned; 0 = default)
  int batch_refs = 0;       // live batches holding this plan (their groups fix row_nr / conv_nc)
  size_t esz = 8;
  int64_t P = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  // device buffers
  void* X = nullptr;        // x-spectral intermediate [B][M_x/cb][rows][cb]
  void* xcur = nullptr;     // intermediate the passes work on (X, or the adjoint state)
  void* Xadj = nullptr;     // second intermediate (adjoint state while the forward is recomputed)
  size_t X_bytes = 0;
  void* Yb = nullptr;       // 3D y-spectral intermediate [B][M_x/cb][M_y][N_z][cb]
  void* kc = nullptr;       // Kahan compensation [B][P] as bf16 (re, im) pairs (C64)
  size_t kc_bytes = 0;      // its size, rounded up to 8 bytes
  void* ghat = nullptr;     // folded spectrum
  int64_t ghat_n = 0;
  void* tw[3] = {nullptr, nullptr, nullptr};
  double* partials = nullptr;
  size_t partials_cap = 0;  // doubles
  double* resid = nullptr;
  size_t resid_cap = 0;
  void* pstore = nullptr;   // adjoint: stored forward partial sums
  size_t pstore_bytes = 0;
  void* ckpt = nullptr;     // adjoint recompute: checkpoints
  size_t ckpt_bytes = 0;
  double* jpart = nullptr;
  size_t jpart_cap = 0;
  int64_t device_bytes = 0;
  bool green_ready = false;
  // density contrast (2D padded plans): caller's float64 [N_y][N_x] map, and
  // the term kept in space between the two row passes of a term
  const double* gamma = nullptr;
  void* ubuf = nullptr;
  size_t ubuf_bytes = 0;
  // periodic (unpadded) plans of the paper's own scheme
  bool periodic = false;
  void* ghat_vv = nullptr;  // g~ VV (Case II k-space potential) or NULL
  double eps = 0.0;         // the shift of the periodic spectrum
  void* psi0 = nullptr;     // [B][P] G s of the current iteration
  int* iflags = nullptr;    // device {done, iterations}
  double* ierrs = nullptr;  // device error history
  size_t ierrs_cap = 0;
  std::string err;
  // per-pass event timing
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<std::pair<int, size_t>> ev_marks;  // (kind, index of the start event)
};

namespace {

thread_local std::string g_create_err;

int fail(tbs_plan* p, int code, const std::string& msg) {
  if (p) p->err = msg;
  else g_create_err = msg;
  return code;
}

int hip_fail(tbs_plan* p, hipError_t e, const char* what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return fail(p, TBS_ERR_HIP, m);
}

#define TBS_HIP(plan, call)                              \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return hip_fail(plan, e_, #call); \
  } while (0)

#define TBS_LAUNCH(plan, call)                                              \
  do {                                                                      \
    int e_ = (call);                                                        \
    if (e_ != 0) return hip_fail(plan, (hipError_t)e_, #call);               \
  } while (0)

int dev_alloc(tbs_plan* p, void** ptr, size_t bytes) {
  if (bytes == 0) {
    *ptr = nullptr;
    return TBS_OK;
  }
  hipError_t e = hipMalloc(ptr, bytes);
  if (e != hipSuccess) {
    *ptr = nullptr;
    (void)hipGetLastError();
    return fail(p, e == hipErrorOutOfMemory ? TBS_ERR_OOM : TBS_ERR_HIP,
                "device allocation of " + std::to_string(bytes) + " bytes failed: " +
                    hipGetErrorString(e));
  }
  p->device_bytes += (int64_t)bytes;
  return TBS_OK;
}

void dev_free(tbs_plan* p, void*& ptr, size_t bytes) {
  if (ptr) {
    (void)hipFree(ptr);
    p->device_bytes -= (int64_t)bytes;
  }
  ptr = nullptr;
}

bool is_fin(double v) { return std::isfinite(v); }

// Twiddle table of one FFT length in the stage layout of tbs_fft.hpp, built in
// extended precision and rounded once.
std::vector<zd> twiddles(int M, bool fp64) {
  const int E = tbs::fft_elems_per_thread(M, fp64);
  const tbs::Stages st = tbs::make_stages(M, E);
  std::vector<zd> out;
  out.reserve(M);
  long L = 1;
  for (int s = 0; s < st.n; ++s) {
    const long R = st.r[s];
    for (long r = 1; r < R; ++r)
      for (long k = 0; k < L; ++k) {
        const long den = L * R;
        const long num = (r * k) % den;
        const long double ang = 2.0L * 3.141592653589793238462643383279502884L * (long double)num /
                                (long double)den;
        out.push_back(zd{(double)cosl(ang), (double)(-sinl(ang))});  // e^{-i ang}
      }
    L *= R;
  }
  return out;
}

int upload_twiddles(tbs_plan* p, int M, bool fp64, void** dst) {
  std::vector<zd> t = twiddles(M, fp64);
  size_t bytes = t.size() * (fp64 ? 16 : 8);
  if (bytes == 0) bytes = 16;
  int rc = dev_alloc(p, dst, bytes);
  if (rc) return rc;
  if (fp64) {
    TBS_HIP(p, hipMemcpy(*dst, t.data(), t.size() * 16, hipMemcpyHostToDevice));
  } else {
    std::vector<float> f(2 * t.size());
    for (size_t i = 0; i < t.size(); ++i) {
      f[2 * i] = (float)t[i].re;
      f[2 * i + 1] = (float)t[i].im;
    }
    TBS_HIP(p, hipMemcpy(*dst, f.data(), f.size() * 4, hipMemcpyHostToDevice));
  }
  return TBS_OK;
}

int ensure_doubles(tbs_plan* p, double** buf, size_t* cap, size_t need) {
  if (*cap >= need) return TBS_OK;
  void* q = *buf;
  dev_free(p, q, *cap * 8);
  *buf = nullptr;
  *cap = 0;
  int rc = dev_alloc(p, &q, need * 8);
  if (rc) return rc;
  *buf = (double*)q;
  *cap = need;
  return TBS_OK;
}

enum { PK_ROW_FIRST = 0, PK_ROW_MID = 1, PK_ROW_LAST = 2, PK_COL_CONV = 3, PK_COL_FWD = 4,
       PK_COL_INV = 5, PK_N = 6 };

hipEvent_t next_event(tbs_plan* p) {
  if (p->ev_used == p->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    p->ev_pool.push_back(e);
  }
  return p->ev_pool[p->ev_used++];
}

// Bracket a launch with events when profiling.
struct ProfScope {
  tbs_plan* p;
  hipEvent_t e1 = nullptr;
  ProfScope(tbs_plan* pl, int kind) : p(pl) {
    if (!p->prof) return;
    const size_t idx = p->ev_used;
    hipEvent_t e0 = next_event(p);
    e1 = next_event(p);
    if (!e0 || !e1) {
      e1 = nullptr;
      return;
    }
    (void)hipEventRecord(e0, p->stream);
    p->ev_marks.push_back({kind, idx});
  }
  ~ProfScope() {
    if (e1) (void)hipEventRecord(e1, p->stream);
  }
};

int row_blocks(const tbs_plan* p) {
  const int NR = p->row_nr ? p->row_nr : tbs::row_rows_per_block((int)p->M[0], p->fp64);
  const int64_t rows = p->N[1] * p->N[2];
  return (int)((rows + NR - 1) / NR);
}

// Arguments of one row pass.
tbs::RowArgs make_row_args(tbs_plan* p, int in_mode, int acc, int out_spec, bool adjoint,
                           const void* src, const void* V, void* pacc, void* pstore_slot,
                           const void* pair, void* grad, double* partials) {
  tbs::RowArgs a{};
  a.X = p->xcur;
  a.src = src;
  a.V = V;
  a.p = pacc;
  a.c = p->kc;
  a.pair = pair;
  a.grad = grad;
  a.partials = partials;
  a.tw = p->tw[0];
  a.nx = (int)p->N[0];
  a.ny = (int)p->N[1];
  a.nz = (int)p->N[2];
  a.nrows = (int)(p->N[1] * p->N[2]);
  a.nrhs = p->batch;
  a.in_mode = in_mode;
  a.acc = acc;
  a.out_spec = out_spec;
  a.conj_v = adjoint ? 1 : 0;
  a.pstore = pstore_slot;
  a.cb = p->cb;
  a.xcd_remap = 1;
  return a;
}

// Row pass of one term.
int run_row(tbs_plan* p, int in_mode, int acc, int out_spec, bool adjoint, const void* src,
            const void* V, void* pacc, void* pstore_slot, const void* pair, void* grad,
            double* partials) {
  const tbs::RowArgs a = make_row_args(p, in_mode, acc, out_spec, adjoint, src, V, pacc,
                                       pstore_slot, pair, grad, partials);
  ProfScope ps(p, in_mode == tbs::ROW_IN_SOURCE ? PK_ROW_FIRST : (out_spec ? PK_ROW_MID : PK_ROW_LAST));
  TBS_LAUNCH(p, tbs::launch_row_pass(p->fp64, (int)p->M[0], a, row_blocks(p), p->row_nr, p->stream));
  return TBS_OK;
}

// Row pass with prepared arguments.
int run_row_args(tbs_plan* p, const tbs::RowArgs& a, int kind) {
  ProfScope ps(p, kind);
  TBS_LAUNCH(p, tbs::launch_row_pass(p->fp64, (int)p->M[0], a, row_blocks(p), p->row_nr, p->stream));
  return TBS_OK;
}

// Arguments of the 2D column convolution pass; *nc receives the columns per block.
tbs::ColArgs make_conv2d_args(tbs_plan* p, bool adjoint, int* nc) {
  const int64_t cb = p->cb;
  const int64_t nkb = p->M[0] / cb;
  tbs::ColArgs a{};
  a.in = p->xcur;
  a.out = p->xcur;
  a.tw = p->tw[1];
  a.ghat = p->ghat;
  a.op = tbs::COL_CONV;
  a.conj_g = adjoint ? 1 : 0;
  a.n_in = (int)p->N[1];
  a.n_out = (int)p->N[1];
  a.in_astride = a.out_astride = cb;
  a.in_rs = a.out_rs = nkb * p->N[1] * cb;
  a.in_s1 = a.out_s1 = p->N[1] * cb;
  a.in_s0 = a.out_s0 = 0;
  *nc = p->conv_nc ? p->conv_nc : tbs::conv_cols_per_block((int)p->M[1], p->fp64, (int)cb);
  a.nrhs = p->batch;
  a.sub = (int)cb / *nc;
  a.n1 = (int)nkb * a.sub;
  a.n0 = 1;
  a.cb = (int)cb;
  a.zcols = 0;
  a.zlim = 1;
  a.mx = (int)p->M[0];
  a.mm = 1;
  a.g_sx = p->M[1] / 2 + 1;
  a.g_sm = 0;
  a.xcd_remap = 1;
  a.mirror = 1;
  return a;
}

// Green's-function application to the row-pass output (all columns).
int run_cols(tbs_plan* p, bool adjoint) {
  const int64_t cb = p->cb;
  const int64_t nkb = p->M[0] / cb;
  if (p->ndim == 2) {
    int nc = 0;
    const tbs::ColArgs a = make_conv2d_args(p, adjoint, &nc);
    ProfScope ps(p, PK_COL_CONV);
    TBS_LAUNCH(p, tbs::launch_col_pass(p->fp64, (int)p->M[1], nc, a, p->stream));
    return TBS_OK;
  }
  // 3D: y forward (A -> B), z convolution (in B), y inverse (B -> A).
  const int64_t ny = p->N[1], nz = p->N[2], my = p->M[1];
  const int NZ = my <= 512 ? 4 : 1;  // z planes per y-pass block (LDS-bound)
  const int NC = NZ * (int)cb;
  const int nzb = (int)((nz + NZ - 1) / NZ);
  tbs::ColArgs y{};
  y.sub = 1;
  y.tw = p->tw[1];
  y.nrhs = p->batch;
  y.n1 = (int)nkb;
  y.n0 = nzb;
  y.cb = (int)cb;
  y.zcols = NZ;
  y.zlim = (int)nz;
  y.xcd_remap = 1;
  // A element (rhs, kxb, y, z, c): ((rhs*nkb + kxb)*ny + y)*nz*cb + z*cb + c
  // B element (rhs, kxb, ky, z, c): ((rhs*nkb + kxb)*my + ky)*nz*cb + z*cb + c
  tbs::ColArgs f = y;
  f.in = p->xcur;
  f.out = p->Yb;
  f.op = tbs::COL_FWD;
  f.n_in = (int)ny;
  f.n_out = (int)my;
  f.in_astride = nz * cb;
  f.out_astride = nz * cb;
  f.in_rs = nkb * ny * nz * cb;
  f.in_s1 = ny * nz * cb;
  f.in_s0 = NZ * cb;
  f.out_rs = nkb * my * nz * cb;
  f.out_s1 = my * nz * cb;
  f.out_s0 = NZ * cb;
  {
    ProfScope ps(p, PK_COL_FWD);
    TBS_LAUNCH(p, tbs::launch_col_pass(p->fp64, (int)my, NC, f, p->stream));
  }

  tbs::ColArgs z{};
  // z lines per block: the tuned count (a divisor of the layout block) or cb
  const int znc = p->conv_nc ? p->conv_nc : (int)cb;
  z.sub = (int)cb / znc;
  z.in = p->Yb;
  z.out = p->Yb;
  z.tw = p->tw[2];
  z.ghat = p->ghat;
  z.op = tbs::COL_CONV;
  z.conj_g = adjoint ? 1 : 0;
  z.n_in = (int)nz;
  z.n_out = (int)nz;
  z.in_astride = z.out_astride = cb;
  z.in_rs = z.out_rs = nkb * my * nz * cb;
  z.in_s1 = z.out_s1 = my * nz * cb;
  z.in_s0 = z.out_s0 = nz * cb;
  z.nrhs = p->batch;
  z.n1 = (int)nkb * z.sub;
  z.n0 = (int)my;
  z.cb = (int)cb;
  z.zcols = 0;
  z.zlim = 1;
  z.mx = (int)p->M[0];
  z.mm = (int)my;
  z.g_sx = (p->M[1] / 2 + 1) * (p->M[2] / 2 + 1);
  z.g_sm = p->M[2] / 2 + 1;
  z.xcd_remap = 1;
  z.mirror = 1;
  {
    ProfScope ps(p, PK_COL_CONV);
    TBS_LAUNCH(p, tbs::launch_col_pass(p->fp64, (int)p->M[2], znc, z, p->stream));
  }

  tbs::ColArgs iv = y;
  iv.in = p->Yb;
  iv.out = p->xcur;
  iv.op = tbs::COL_INV;
  iv.n_in = (int)my;
  iv.n_out = (int)ny;
  iv.in_astride = nz * cb;
  iv.out_astride = nz * cb;
  iv.in_rs = nkb * my * nz * cb;
  iv.in_s1 = my * nz * cb;
  iv.in_s0 = NZ * cb;
  iv.out_rs = nkb * ny * nz * cb;
  iv.out_s1 = ny * nz * cb;
  iv.out_s0 = NZ * cb;
  {
    ProfScope ps(p, PK_COL_INV);
    TBS_LAUNCH(p, tbs::launch_col_pass(p->fp64, (int)my, NC, iv, p->stream));
  }
  return TBS_OK;
}

int check_residuals(tbs_plan* p, double* residual_out, int nterms) {
  TBS_HIP(p, hipMemcpyAsync(residual_out, p->resid, sizeof(double) * p->batch * nterms,
                            hipMemcpyDeviceToHost, p->stream));
  TBS_HIP(p, hipStreamSynchronize(p->stream));
  int warn = TBS_OK;
  for (int b = 0; b < p->batch; ++b) {
    const double* r = residual_out + (size_t)b * nterms;
    int grow = 0;
    for (int n = 0; n < nterms; ++n) {
      if (!is_fin(r[n])) {
        p->err = "non-finite residual (non-finite source or potential?)";
        return TBS_WARN_NONFINITE;
      }
      grow = (n > 0 && r[n] > r[n - 1]) ? grow + 1 : 0;
      if (grow >= 3 && warn == TBS_OK) {
        p->err = "residuals grew over 3 consecutive terms (series diverging: rho(GV) >= 1?)";
        warn = TBS_WARN_DIVERGING;
      }
    }
  }
  return warn;
}

// Forward series.  pstore (optional): slot K-1 receives P_K, K = 1..L-1.
int forward_series(tbs_plan* p, const void* source, const void* V, int L, void* p_out,
                   void* pstore, bool adj = false) {
  const int nblk = row_blocks(p);
  const size_t per_term = (size_t)2 * p->batch * nblk;
  int rc = ensure_doubles(p, &p->partials, &p->partials_cap, per_term * (size_t)L);
  if (rc) return rc;
  rc = ensure_doubles(p, &p->resid, &p->resid_cap, (size_t)p->batch * L);
  if (rc) return rc;
  const size_t slot = (size_t)p->batch * p->P * p->esz;
  const int Leff = (V || p->gamma) ? L : 1;  // V = 0 and no density: u_n = 0 for n >= 1
  // u_0 = G s
  rc = run_row(p, tbs::ROW_IN_SOURCE, tbs::ACC_NONE, 1, adj, source, nullptr, nullptr, nullptr,
               nullptr, nullptr, nullptr);
  if (rc) return rc;
  rc = run_cols(p, adj);
  if (rc) return rc;
  if (p->gamma) {
    // density contrast: each term's field is kept in space, then a second row
    // pass forms V u - div(gamma grad u) (it needs the neighbouring rows)
    if (p->ubuf_bytes < slot) {
      dev_free(p, p->ubuf, p->ubuf_bytes);
      p->ubuf_bytes = 0;
      rc = dev_alloc(p, &p->ubuf, slot);
      if (rc) return rc;
      p->ubuf_bytes = slot;
    }
    for (int n = 1; n <= L; ++n) {
      void* st = (pstore && n < L) ? (void*)((char*)pstore + (size_t)(n - 1) * slot) : nullptr;
      tbs::RowArgs a = make_row_args(p, tbs::ROW_IN_SPECTRAL, n == 1 ? tbs::ACC_INIT : tbs::ACC_ADD, 0,
                                     false, nullptr, nullptr, p_out, st, nullptr, nullptr,
                                     p->partials + (size_t)(n - 1) * per_term);
      a.ustore = n < L ? p->ubuf : nullptr;
      rc = run_row_args(p, a, n < L ? PK_ROW_MID : PK_ROW_LAST);
      if (rc) return rc;
      if (n == L) break;
      tbs::RowArgs b = make_row_args(p, tbs::ROW_IN_SPATIAL, tbs::ACC_NONE, 1, false, p->ubuf, V,
                                     nullptr, nullptr, nullptr, nullptr, nullptr);
      b.gamma = p->gamma;
      b.inv_dx2 = 1.0 / (p->dx * p->dx);
      rc = run_row_args(p, b, PK_ROW_FIRST);
      if (rc) return rc;
      rc = run_cols(p, false);
      if (rc) return rc;
    }
    TBS_LAUNCH(p, tbs::launch_finish_norms(p->partials, L, L, p->batch, nblk, p->resid, p->stream));
    return TBS_OK;
  }
  for (int n = 1; n < Leff; ++n) {
    void* st = pstore ? (void*)((char*)pstore + (size_t)(n - 1) * slot) : nullptr;
    rc = run_row(p, tbs::ROW_IN_SPECTRAL, n == 1 ? tbs::ACC_INIT : tbs::ACC_ADD, 1, adj,
                 nullptr, V, p_out, st, nullptr, nullptr, p->partials + (size_t)(n - 1) * per_term);
    if (rc) return rc;
    rc = run_cols(p, adj);
    if (rc) return rc;
  }
  rc = run_row(p, tbs::ROW_IN_SPECTRAL, Leff == 1 ? tbs::ACC_INIT : tbs::ACC_ADD, 0, adj,
               nullptr, nullptr, p_out, nullptr, nullptr, nullptr,
               p->partials + (size_t)(Leff - 1) * per_term);
  if (rc) return rc;
  // terms n >= Leff are exactly zero (V = 0)
  TBS_LAUNCH(p, tbs::launch_finish_norms(p->partials, L, Leff, p->batch, nblk, p->resid, p->stream));
  return TBS_OK;
}

// ---------------------------------------------------------- tuning cache --
// Block shapes chosen by the tuners, per device model and problem shape, kept
// for the life of the process and, when the environment variable
// TBS_TUNE_CACHE names a file, read from it on first use and appended to on
// every new choice (one "key = values" line per choice; later lines win).
struct TuneCache {
  std::mutex mu;
  bool loaded = false;
  std::map<std::string, std::vector<int>> entries;
};

TuneCache& tune_cache() {
  static TuneCache c;
  return c;
}

std::string device_tag(int device) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
    (void)hipGetLastError();
    return "device" + std::to_string(device);
  }
  std::string arch = prop.gcnArchName;
  for (char& ch : arch)
    if (ch == ' ' || ch == '=') ch = '_';
  return arch + "/" + std::to_string(prop.multiProcessorCount) + "cu";
}

void tune_cache_load(TuneCache& c) {  // caller holds c.mu
  if (c.loaded) return;
  c.loaded = true;
  const char* path = std::getenv("TBS_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char line[4096];
  while (std::fgets(line, sizeof line, f)) {
    const std::string sl(line);
    const size_t eq = sl.find(" = ");
    if (eq == std::string::npos) continue;
    std::vector<int> vals;
    const char* q = sl.c_str() + eq + 3;
    while (true) {
      char* end = nullptr;
      const long v = std::strtol(q, &end, 10);
      if (end == q) break;
      vals.push_back((int)v);
      q = end;
    }
    if (!vals.empty()) c.entries[sl.substr(0, eq)] = vals;
  }
  std::fclose(f);
}

bool tune_lookup(const std::string& key, std::vector<int>* vals) {
  TuneCache& c = tune_cache();
  std::lock_guard<std::mutex> g(c.mu);
  tune_cache_load(c);
  auto it = c.entries.find(key);
  if (it == c.entries.end()) return false;
  *vals = it->second;
  return true;
}

void tune_store(const std::string& key, const std::vector<int>& vals) {
  TuneCache& c = tune_cache();
  std::lock_guard<std::mutex> g(c.mu);
  tune_cache_load(c);
  c.entries[key] = vals;
  const char* path = std::getenv("TBS_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::string line = key + " =";
  for (int v : vals) line += " " + std::to_string(v);
  line += "\n";
  std::fputs(line.c_str(), f);
  std::fclose(f);
}

bool in_list(int v, const int* list, int n) {
  for (int i = 0; i < n; ++i)
    if (list[i] == v) return true;
  return false;
}

int check_plan_ready(tbs_plan* p) {
  if (!p) return TBS_ERR_INVALID;
  if (p->periodic)
    return fail(p, TBS_ERR_STATE, "periodic plans run tbs_iterate only");
  if (!p->green_ready)
    return fail(p, TBS_ERR_STATE, "the Green spectrum is not set: call tbs_green_tabulate first");
  return TBS_OK;
}

}  // namespace

// ------------------------------------------------------- static workspace --
// tbs_solve_noalloc keeps the series' workspace in this file-scope device
// array: one copy per GPU, held until the process ends.  In host code the
// array's name only stands in for the device symbol; its device address is
// taken once per device with hipGetSymbolAddress and used from then on.
#define TBS_SCRATCH_BYTES (128ull << 20)
static __device__ __align__(256) unsigned char scratch[TBS_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the scratch array on the plan's device (looked up on the
// first call for that device, with that device current).
int scratch_address(tbs_plan* p, void** out) {
  if (p->device < 0 || p->device >= kMaxDevices)
    return fail(p, TBS_ERR_UNSUPPORTED, "device index beyond the static workspace table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[p->device]) {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(p, e, "hipGetDevice");
    if (cur != p->device && (e = hipSetDevice(p->device)) != hipSuccess) return hip_fail(p, e, "hipSetDevice");
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != p->device) (void)hipSetDevice(cur);
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return hip_fail(p, e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    }
    g_scratch_ptr[p->device] = ptr;
  }
  *out = g_scratch_ptr[p->device];
  return TBS_OK;
}

size_t align256(size_t n) { return (n + 255) / 256 * 256; }

}  // namespace

// ------------------------------------------------------------- batches ----

struct tbs_batch {
  std::vector<tbs_plan*> plans;
  hipStream_t stream = nullptr;   // the batch's own stream (graphs are recorded and run here)
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  bool fp64 = false;
  // Launch chains: pass sequences on their own streams, so that one chain's
  // launches fill the CUs the others' leave idle at their ends: the tiles of
  // each set go to the chains in turn (with one set of whole plans, the plans
  // split into parts of equal work), and the sets still run one after the
  // other (fork and join per set), so the cache holds one set.
  int chains = 1;
  hipStream_t cstream[kMaxChains] = {};  // chain c > 0 runs on cstream[c]
  hipEvent_t ev_fork = nullptr;          // per set: the other chains start
  hipEvent_t ev_join[kMaxChains] = {};   // per set: chain c has ended
  // Tiles: a plan's right-hand sides [r0, r0 + nrhs).  Sets: tiles whose
  // working set (intermediate, sum, compensation, potential, spectrum) fits
  // the device's last-level cache together; the series runs set by set (all
  // terms of one set, then the next), so that each set's data stays in the
  // 256 MB Infinity Cache between passes instead of streaming through HBM.
  struct Tile {
    int plan = 0, r0 = 0, nrhs = 0, set = 0, chain = 0;
  };
  std::vector<Tile> tiles;
  int nsets = 1;
  int tile_rhs = 0, cache_mb = 0;  // the tiling the sets were made with (0: whole plans, one set)
  struct Group {
    int chain = 0, set = 0;
    int M = 0, cb = 4, nc = 0, nr = 0;
    std::vector<int> members;  // tile indices
    int first = 0;             // index of the first member in the descriptor order
    int starts_off = 0;        // offset of this group's starts array
    int total = 0;             // blocks of one grouped launch
  };
  std::vector<Group> rgroups, cgroups;
  std::vector<int> rpos, cpos;   // tile -> position in the row / column descriptor order
  std::vector<int> chain_of;     // plan -> chain
  // device tables
  void* d_row = nullptr;         // RowArgs [L+1][ntiles]
  size_t d_row_bytes = 0;
  void* d_col = nullptr;         // ColArgs [ntiles]
  void* d_starts = nullptr;      // int
  size_t d_starts_bytes = 0;
  // descriptor tables and the arguments they were built for; the recorded graph
  bool tables_ready = false;
  hipGraphExec_t exec = nullptr;
  bool counted = false;          // batch_refs of the plans incremented
  std::vector<const void*> key;
  int key_L = 0;
  // per-launch event timing (tbs_batch_profile_*): entry 3 g + mode for row
  // group g (mode 0 first, 1 middle, 2 last row pass), 3 nrg + g for column
  // group g; marks hold (entry, index of the start event in the pool)
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<std::pair<int, size_t>> marks;
  std::vector<double> prof_ms;
  std::vector<int64_t> prof_n;
  std::string err;
};

namespace {

int bfail(tbs_batch* b, int code, const std::string& m) {
  if (b) b->err = m;
  return code;
}

void batch_free_tables(tbs_batch* b) {
  if (b->d_row) (void)hipFree(b->d_row);
  if (b->d_col) (void)hipFree(b->d_col);
  if (b->d_starts) (void)hipFree(b->d_starts);
  b->d_row = b->d_col = b->d_starts = nullptr;
  b->d_row_bytes = b->d_starts_bytes = 0;
}

void batch_drop_graph(tbs_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  b->exec = nullptr;
  b->tables_ready = false;
  b->key.clear();
  b->key_L = 0;
}

// Working set of a tile of nrhs right-hand sides of plan p (bytes the passes
// of one term touch): intermediate, sum and compensation per right-hand side,
// the potential and the folded spectrum once.
double tile_bytes(const tbs_plan* p, int nrhs) {
  const double P = (double)p->P, esz = (double)p->esz;
  return nrhs * ((double)p->N[1] * p->M[0] * esz + P * (esz + (p->fp64 ? 0.0 : 4.0))) + P * esz +
         (double)(p->M[0] / 2 + 1) * (p->M[1] / 2 + 1) * esz;
}

// Split the plans into tiles of at most TBS_BATCH_TILE_RHS right-hand sides
// (default 2) and pack consecutive tiles into sets of at most
// TBS_BATCH_CACHE_MB megabytes of working set (default 280; 0: one set of
// whole plans).  The estimate counts each tile's potential and spectrum, which
// tiles of one plan in a set share: 280 MB of it holds three tiles of the
// smaller 2560-line grids, about 225 MB of distinct data for the 256 MB cache.  The tiles of a set go to the launch chains in turn.
void batch_tile(tbs_batch* b) {
  const int nplans = (int)b->plans.size();
  double cap = 280e6;
  int trhs = TBS_BATCH_TILE_RHS_DEFAULT;
  if (const char* e = std::getenv("TBS_BATCH_CACHE_MB")) cap = std::atof(e) * 1e6;
  if (const char* e = std::getenv("TBS_BATCH_TILE_RHS")) trhs = std::max(1, std::atoi(e));
  b->tiles.clear();
  if (!(cap > 0)) {
    for (int i = 0; i < nplans; ++i) b->tiles.push_back({i, 0, b->plans[i]->batch, 0, b->chain_of[i]});
    b->nsets = 1;
    b->tile_rhs = b->cache_mb = 0;
    return;
  }
  b->tile_rhs = trhs;
  b->cache_mb = (int)(cap / 1e6 + 0.5);
  int set = 0;
  double acc = 0.0;
  bool empty = true;
  int in_set = 0;  // tiles already in the current set
  for (int i = 0; i < nplans; ++i) {
    const tbs_plan* p = b->plans[i];
    for (int r0 = 0; r0 < p->batch; r0 += trhs) {
      const int nr = std::min(trhs, p->batch - r0);
      const double w = tile_bytes(p, nr);
      if (!empty && acc + w > cap) {
        ++set;
        acc = 0.0;
        in_set = 0;
      }
      b->tiles.push_back({i, r0, nr, set, in_set % b->chains});
      ++in_set;
      acc += w;
      empty = false;
    }
  }
  b->nsets = set + 1;
}

// Group the batch's tiles by set, padded length and block shape (rows: M_x
// and rows per block; columns: M_y, layout block and columns per block) and
// upload the block offsets of every group; called again after the shapes
// change.
int batch_group(tbs_batch* b) {
  batch_tile(b);
  // TBS_BATCH_SHAPE="nr,nc": rows and columns per block for the plans the
  // tuners have not set, where the length has that shape (a check that every
  // block shape gives the same results)
  if (const char* e = std::getenv("TBS_BATCH_SHAPE")) {
    int fnr = 0, fnc = 0;
    if (std::sscanf(e, "%d,%d", &fnr, &fnc) == 2) {
      for (tbs_plan* p : b->plans) {
        int cand[8];
        if (!p->row_nr && in_list(fnr, cand, tbs::row_nr_candidates((int)p->M[0], p->fp64, cand)))
          p->row_nr = fnr;
        if (!p->conv_nc && in_list(fnc, cand, tbs::conv_nc_candidates((int)p->M[1], p->fp64, p->cb, cand)))
          p->conv_nc = fnc;
      }
    }
  }
  const int nt = (int)b->tiles.size();
  b->rgroups.clear();
  b->cgroups.clear();
  b->rpos.assign(nt, 0);
  b->cpos.assign(nt, 0);
  auto find_or_add = [](std::vector<tbs_batch::Group>& gs, int set, int chain, int M, int cb, int nc,
                        int nr) -> tbs_batch::Group& {
    for (auto& g : gs)
      if (g.set == set && g.chain == chain && g.M == M && g.cb == cb && g.nc == nc && g.nr == nr) return g;
    gs.push_back(tbs_batch::Group());
    gs.back().set = set;
    gs.back().chain = chain;
    gs.back().M = M;
    gs.back().cb = cb;
    gs.back().nc = nc;
    gs.back().nr = nr;
    return gs.back();
  };
  for (int t = 0; t < nt; ++t) {
    const tbs_batch::Tile& tl = b->tiles[t];
    tbs_plan* p = b->plans[tl.plan];
    const int chain = tl.chain;
    const int nr = p->row_nr ? p->row_nr : tbs::row_rows_per_block((int)p->M[0], p->fp64);
    find_or_add(b->rgroups, tl.set, chain, (int)p->M[0], p->cb, 0, nr).members.push_back(t);
    int nc = 0;
    (void)make_conv2d_args(p, false, &nc);
    find_or_add(b->cgroups, tl.set, chain, (int)p->M[1], p->cb, nc, 0).members.push_back(t);
  }
  std::vector<int> starts;
  int pos = 0;
  for (auto& g : b->rgroups) {
    g.first = pos;
    g.starts_off = (int)starts.size();
    int acc = 0;
    for (int t : g.members) {
      b->rpos[t] = pos++;
      starts.push_back(acc);
      acc += row_blocks(b->plans[b->tiles[t].plan]) * b->tiles[t].nrhs;
    }
    g.total = acc;
  }
  pos = 0;
  for (auto& g : b->cgroups) {
    g.first = pos;
    g.starts_off = (int)starts.size();
    int acc = 0;
    for (int t : g.members) {
      b->cpos[t] = pos++;
      starts.push_back(acc);
      int nc = 0;
      const tbs::ColArgs c = make_conv2d_args(b->plans[b->tiles[t].plan], false, &nc);
      acc += b->tiles[t].nrhs * c.n1 * c.n0;
    }
    g.total = acc;
  }
  if (b->d_starts) (void)hipFree(b->d_starts);
  b->d_starts = nullptr;
  b->d_starts_bytes = starts.size() * sizeof(int);
  if (hipMalloc(&b->d_starts, b->d_starts_bytes) != hipSuccess ||
      hipMemcpy(b->d_starts, starts.data(), b->d_starts_bytes, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipGetLastError();
    return TBS_ERR_OOM;
  }
  return TBS_OK;
}

// Arguments of tile t's row pass of term n (0: the source in; L: the last)
// and of its column convolution: the plan's arguments with every per-RHS
// array moved to the tile's first right-hand side.
tbs::RowArgs tile_row_args(tbs_batch* b, int t, int n, int L, const void* source, const void* V,
                           void* p_out) {
  const tbs_batch::Tile& tl = b->tiles[t];
  tbs_plan* p = b->plans[tl.plan];
  const int nblk = row_blocks(p);
  const size_t per_term = (size_t)2 * p->batch * nblk;
  const size_t sp = (size_t)tl.r0 * p->P;                        // [rhs][P] values
  const size_t xs = (size_t)tl.r0 * p->M[0] * p->N[1] * p->N[2];  // [rhs][kxb][rows][cb] values
  tbs::RowArgs r;
  if (n == 0)
    r = make_row_args(p, tbs::ROW_IN_SOURCE, tbs::ACC_NONE, 1, false, (const char*)source + sp * p->esz,
                      nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
  else
    r = make_row_args(p, tbs::ROW_IN_SPECTRAL, n == 1 ? tbs::ACC_INIT : tbs::ACC_ADD, n < L ? 1 : 0, false,
                      nullptr, V, (char*)p_out + sp * p->esz, nullptr, nullptr, nullptr,
                      p->partials + (size_t)(n - 1) * per_term + (size_t)2 * tl.r0 * nblk);
  r.X = (char*)p->X + xs * p->esz;
  if (r.c) r.c = (char*)r.c + sp * 4;
  r.nrhs = tl.nrhs;
  return r;
}

tbs::ColArgs tile_col_args(tbs_batch* b, int t) {
  const tbs_batch::Tile& tl = b->tiles[t];
  tbs_plan* p = b->plans[tl.plan];
  const size_t xs = (size_t)tl.r0 * p->M[0] * p->N[1] * p->N[2];
  int nc = 0;
  tbs::ColArgs c = make_conv2d_args(p, false, &nc);
  c.in = (const char*)p->X + xs * p->esz;
  c.out = (char*)p->X + xs * p->esz;
  c.nrhs = tl.nrhs;
  return c;
}

// Start event of a profiled launch (entry e); returns the end event to record
// after the launch, or nullptr when not profiling (or out of events).
hipEvent_t batch_prof_begin(tbs_batch* b, int e, hipStream_t s) {
  if (!b->prof) return nullptr;
  while (b->ev_used + 2 > b->ev_pool.size()) {
    hipEvent_t ev;
    if (hipEventCreate(&ev) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    b->ev_pool.push_back(ev);
  }
  const size_t idx = b->ev_used;
  b->ev_used += 2;
  if (hipEventRecord(b->ev_pool[idx], s) != hipSuccess) return nullptr;
  b->marks.push_back({e, idx});
  return b->ev_pool[idx + 1];
}

// Waits for the batch stream and the chains' streams; false on a failed solve.
bool batch_sync(tbs_batch* b) {
  bool ok = !b->stream || hipStreamSynchronize(b->stream) == hipSuccess;
  for (int c = 1; c < kMaxChains; ++c)
    if (b->cstream[c] && hipStreamSynchronize(b->cstream[c]) != hipSuccess) ok = false;
  return ok;
}

// Enqueue the whole batched series (no synchronisation).  With several
// chains each set's chains c > 0 run on their own streams, forked from the
// batch stream at the start of the set and joined back at its end.
int batch_enqueue(tbs_batch* b, int L) {
  const int nt = (int)b->tiles.size();
  const tbs::RowArgs* drow = (const tbs::RowArgs*)b->d_row;
  const tbs::ColArgs* dcol = (const tbs::ColArgs*)b->d_col;
  const int* dst = (const int*)b->d_starts;
  const int nrg = (int)b->rgroups.size();
  auto rows = [&](int chain, int set, int n, hipStream_t s) -> int {
    for (int gi = 0; gi < nrg; ++gi) {
      const auto& g = b->rgroups[gi];
      if (g.chain != chain || g.set != set) continue;
      hipEvent_t end = batch_prof_begin(b, 3 * gi + (n == 0 ? 0 : (n == L ? 2 : 1)), s);
      int e = tbs::launch_row_group(b->fp64, g.M, g.cb, g.nr, drow + (size_t)n * nt + g.first,
                                    dst + g.starts_off, (int)g.members.size(), g.total, s);
      if (e) return bfail(b, TBS_ERR_HIP, std::string("grouped row pass: ") + hipGetErrorString((hipError_t)e));
      if (end && hipEventRecord(end, s) != hipSuccess) return bfail(b, TBS_ERR_HIP, "profile event");
    }
    return TBS_OK;
  };
  auto cols = [&](int chain, int set, hipStream_t s) -> int {
    for (int gi = 0; gi < (int)b->cgroups.size(); ++gi) {
      const auto& g = b->cgroups[gi];
      if (g.chain != chain || g.set != set) continue;
      hipEvent_t end = batch_prof_begin(b, 3 * nrg + gi, s);
      int e = tbs::launch_col_group(b->fp64, g.M, g.nc, dcol + g.first, dst + g.starts_off,
                                    (int)g.members.size(), g.total, s);
      if (e) return bfail(b, TBS_ERR_HIP, std::string("grouped column pass: ") + hipGetErrorString((hipError_t)e));
      if (end && hipEventRecord(end, s) != hipSuccess) return bfail(b, TBS_ERR_HIP, "profile event");
    }
    return TBS_OK;
  };
  // one set's series on one chain: the row passes of term n, then (n < L)
  // the column convolutions
  auto set_series = [&](int chain, int set, hipStream_t s) -> int {
    for (int n = 0; n <= L; ++n) {
      int rc = rows(chain, set, n, s);
      if (rc) return rc;
      if (n == L) break;
      rc = cols(chain, set, s);
      if (rc) return rc;
    }
    return TBS_OK;
  };
  // profiled solves run the chains one after the other on one stream, so
  // that every launch's events bracket that launch alone
  const bool many = b->chains > 1 && !b->prof;
  for (int set = 0; set < b->nsets; ++set) {
    if (many && hipEventRecord(b->ev_fork, b->stream) != hipSuccess)
      return bfail(b, TBS_ERR_HIP, "batch chain fork");
    for (int c = 1; many && c < b->chains; ++c)
      if (hipStreamWaitEvent(b->cstream[c], b->ev_fork, 0) != hipSuccess)
        return bfail(b, TBS_ERR_HIP, "batch chain fork");
    for (int c = 0; c < b->chains; ++c) {
      const int rc = set_series(c, set, many && c > 0 ? b->cstream[c] : b->stream);
      if (rc) return rc;
    }
    for (int c = 1; many && c < b->chains; ++c)
      if (hipEventRecord(b->ev_join[c], b->cstream[c]) != hipSuccess ||
          hipStreamWaitEvent(b->stream, b->ev_join[c], 0) != hipSuccess)
        return bfail(b, TBS_ERR_HIP, "batch chain join");
  }
  for (size_t i = 0; i < b->plans.size(); ++i) {
    tbs_plan* p = b->plans[i];
    int e = tbs::launch_finish_norms(p->partials, L, L, p->batch, row_blocks(p), p->resid, b->stream);
    if (e) return bfail(b, TBS_ERR_HIP, std::string("norms: ") + hipGetErrorString((hipError_t)e));
  }
  return TBS_OK;
}

// Adjoint with recomputation: the forward series is run once keeping
// checkpoints (u_{cK}, P_{cK+1}) every K = ceil(sqrt(2L)) terms; the adjoint
// series then walks the segments from last to first, recomputing each
// segment's partial sums from its checkpoint (in the plan's X) while the
// adjoint state waits in a second intermediate.  Memory: 2 ceil((L-1)/K) + K + 1
// fields of [B][P] instead of L.
int adjoint_recompute(tbs_plan* p, const void* source, const void* V, int L, const void* q,
                      void* grad, double* residual_out) {
  const size_t slot = (size_t)p->batch * p->P * p->esz;
  const int K = std::max(1, (int)std::ceil(std::sqrt(2.0 * L)));
  const int C = (L - 2) / K + 1;  // checkpoints at terms 0, K, ..., (C-1)K <= L-2
  const size_t need = slot * (size_t)(2 * C + K + 1);
  if (p->ckpt_bytes < need) {
    dev_free(p, p->ckpt, p->ckpt_bytes);
    p->ckpt_bytes = 0;
    int rc = dev_alloc(p, &p->ckpt, need);
    if (rc) return rc;
    p->ckpt_bytes = need;
  }
  if (!p->Xadj) {
    int rc = dev_alloc(p, &p->Xadj, p->X_bytes);
    if (rc) return rc;
  }
  char* base = (char*)p->ckpt;
  auto ck_u = [&](int c) { return (void*)(base + (size_t)(2 * c) * slot); };
  auto ck_p = [&](int c) { return (void*)(base + (size_t)(2 * c + 1) * slot); };
  auto seg = [&](int j) { return (void*)(base + (size_t)(2 * C + j) * slot); };
  void* pacc = base + (size_t)(2 * C + K) * slot;
  const int nblk = row_blocks(p);
  const size_t per_term = (size_t)2 * p->batch * nblk;
  int rc = ensure_doubles(p, &p->partials, &p->partials_cap, per_term * (size_t)L);
  if (!rc) rc = ensure_doubles(p, &p->resid, &p->resid_cap, (size_t)p->batch * L);
  if (rc) return rc;
  p->xcur = p->X;
  // 1. forward series with checkpoints (and the residuals of every term)
  rc = run_row(p, tbs::ROW_IN_SOURCE, tbs::ACC_NONE, 1, false, source, nullptr, nullptr, nullptr,
               nullptr, nullptr, nullptr);
  if (!rc) rc = run_cols(p, false);
  for (int n = 1; n <= L && !rc; ++n) {
    tbs::RowArgs a = make_row_args(p, tbs::ROW_IN_SPECTRAL, n == 1 ? tbs::ACC_INIT : tbs::ACC_ADD,
                                   n < L ? 1 : 0, false, nullptr, V, pacc, nullptr, nullptr, nullptr,
                                   p->partials + (size_t)(n - 1) * per_term);
    if ((n - 1) % K == 0 && (n - 1) / K < C) {  // term u_{n-1} and P_n are checkpoint c
      a.ustore = ck_u((n - 1) / K);
      a.pstore = ck_p((n - 1) / K);
    }
    rc = run_row_args(p, a, n < L ? PK_ROW_MID : PK_ROW_LAST);
    if (!rc && n < L) rc = run_cols(p, false);
  }
  if (!rc) {
    int e = tbs::launch_finish_norms(p->partials, L, L, p->batch, nblk, p->resid, p->stream);
    if (e) rc = hip_fail(p, (hipError_t)e, "norms");
  }
  if (!rc && residual_out) {
    rc = check_residuals(p, residual_out, L);
    if (rc > 0) rc = TBS_OK;
  }
  if (rc) return rc;
  // 2. adjoint start: w_0 = G^H q into the adjoint state
  p->xcur = p->Xadj;
  rc = run_row(p, tbs::ROW_IN_SOURCE, tbs::ACC_NONE, 1, true, q, nullptr, nullptr, nullptr, nullptr,
               nullptr, nullptr);
  if (!rc) rc = run_cols(p, true);
  p->xcur = p->X;
  // 3. segments from last to first
  for (int c = C - 1; c >= 0 && !rc; --c) {
    const int lo = c * K + 1;               // P_lo is the checkpoint
    const int hi = std::min(c * K + K, L - 1);
    TBS_HIP(p, hipMemcpyAsync(seg(0), ck_p(c), slot, hipMemcpyDeviceToDevice, p->stream));
    if (hi > lo) {
      TBS_HIP(p, hipMemcpyAsync(pacc, ck_p(c), slot, hipMemcpyDeviceToDevice, p->stream));
      if (p->kc) TBS_LAUNCH(p, tbs::launch_zero(p->kc, (int64_t)p->kc_bytes, p->stream));
      tbs::RowArgs a = make_row_args(p, tbs::ROW_IN_SPATIAL, tbs::ACC_NONE, 1, false, ck_u(c), V,
                                     nullptr, nullptr, nullptr, nullptr, nullptr);
      rc = run_row_args(p, a, PK_ROW_FIRST);
      if (!rc) rc = run_cols(p, false);
      for (int n = lo + 1; n <= hi && !rc; ++n) {  // accumulates u_{n-1}: P_n
        tbs::RowArgs b = make_row_args(p, tbs::ROW_IN_SPECTRAL, tbs::ACC_ADD, n < hi ? 1 : 0, false,
                                       nullptr, V, pacc, seg(n - lo), nullptr, nullptr,
                                       p->partials);
        rc = run_row_args(p, b, n < hi ? PK_ROW_MID : PK_ROW_LAST);
        if (!rc && n < hi) rc = run_cols(p, false);
      }
    }
    // adjoint steps pairing with P_hi .. P_lo
    p->xcur = p->Xadj;
    for (int Kp = hi; Kp >= lo && !rc; --Kp) {
      const int m = L - 1 - Kp;
      const bool more = m < L - 2;
      rc = run_row(p, tbs::ROW_IN_SPECTRAL, tbs::ACC_PAIR, more ? 1 : 0, true, nullptr, V, nullptr,
                   nullptr, seg(Kp - lo), grad, p->partials);
      if (!rc && more) rc = run_cols(p, true);
    }
    p->xcur = p->X;
  }
  p->xcur = p->X;
  return rc;
}

}  // namespace

extern "C" {

int tbs_version(void) { return 100; }

const char* tbs_status_string(int s) {
  switch (s) {
    case TBS_OK: return "TBS_OK";
    case TBS_ERR_INVALID: return "TBS_ERR_INVALID";
    case TBS_ERR_UNSUPPORTED: return "TBS_ERR_UNSUPPORTED";
    case TBS_ERR_OOM: return "TBS_ERR_OOM";
    case TBS_ERR_HIP: return "TBS_ERR_HIP";
    case TBS_ERR_STATE: return "TBS_ERR_STATE";
    case TBS_WARN_NONFINITE: return "TBS_WARN_NONFINITE";
    case TBS_WARN_DIVERGING: return "TBS_WARN_DIVERGING";
    case TBS_WARN_NOT_CONVERGED: return "TBS_WARN_NOT_CONVERGED";
    default: return "unknown status";
  }
}

int tbs_padded_length(int64_t n, int padding, int64_t* m_out) {
  if (!m_out || n < 1 || padding < 2 || n > (int64_t)1 << 30) return TBS_ERR_INVALID;
  const int64_t need = padding * n - 1;
  int lens[64];
  const int nl = tbs::fft_supported_lengths(lens, 64);
  for (int i = 0; i < nl; ++i) {
    if (lens[i] >= need) {
      *m_out = lens[i];
      return TBS_OK;
    }
  }
  return TBS_ERR_UNSUPPORTED;
}

int tbs_wavenumber(double omega, double c, double alpha0, double y, tbs_c128* k_out) {
  if (!k_out || !(omega > 0) || !(c > 0) || !(alpha0 >= 0) || !is_fin(y)) return TBS_ERR_INVALID;
  const double a = alpha0 * std::pow(omega, y);
  const double disp = (std::fabs(y - 1.0) < 1e-12) ? 0.0 : std::tan(tbs::kPi * y / 2.0);
  k_out->re = omega / c + a * disp;
  k_out->im = a;
  return TBS_OK;
}

int tbs_background_k0(double omega, double c0, double alpha0, double y, double eps,
                      tbs_c128* k0_out) {
  if (!k0_out || !(eps >= 0)) return TBS_ERR_INVALID;
  tbs_c128 k;
  int rc = tbs_wavenumber(omega, c0, alpha0, y, &k);
  if (rc) return rc;
  const zd k2 = tbs::zadd(tbs::zmul(zd{k.re, k.im}, zd{k.re, k.im}), zd{0.0, eps});
  const zd r = tbs::zsqrt(k2);
  k0_out->re = r.re;
  k0_out->im = r.im;
  return TBS_OK;
}

int tbs_hankel01(tbs_c128 z, tbs_c128* h0, tbs_c128* h1) {
  if (!h0 || !h1 || !(z.re > 0) || !(z.im >= 0)) return TBS_ERR_INVALID;
  zd a, b;
  tbs::hankel01(zd{z.re, z.im}, &a, &b);
  h0->re = a.re;
  h0->im = a.im;
  h1->re = b.re;
  h1->im = b.im;
  return TBS_OK;
}

int tbs_self_cell(int ndim, tbs_c128 k0, double dx, tbs_c128* w0) {
  if (!w0 || !(dx > 0) || !(k0.re > 0) || !(k0.im >= 0)) return TBS_ERR_INVALID;
  zd w;
  if (ndim == 2) w = tbs::self_cell_2d(zd{k0.re, k0.im}, dx);
  else if (ndim == 3) w = tbs::self_cell_3d(zd{k0.re, k0.im}, dx);
  else return TBS_ERR_INVALID;
  w0->re = w.re;
  w0->im = w.im;
  return TBS_OK;
}

void tbs_plan_destroy(tbs_plan* p) {
  if (!p) return;
  (void)hipStreamSynchronize(p->stream);
  dev_free(p, p->X, 0);
  dev_free(p, p->Xadj, 0);
  dev_free(p, p->Yb, 0);
  dev_free(p, p->kc, 0);
  dev_free(p, p->ghat, 0);
  for (auto& t : p->tw) dev_free(p, t, 0);
  void* q = p->partials;
  dev_free(p, q, 0);
  q = p->resid;
  dev_free(p, q, 0);
  dev_free(p, p->pstore, 0);
  dev_free(p, p->ckpt, 0);
  q = p->jpart;
  dev_free(p, q, 0);
  dev_free(p, p->ghat_vv, 0);
  dev_free(p, p->psi0, 0);
  dev_free(p, p->ubuf, 0);
  q = p->iflags;
  dev_free(p, q, 0);
  q = p->ierrs;
  dev_free(p, q, 0);
  for (hipEvent_t e : p->ev_pool) (void)hipEventDestroy(e);
  delete p;
}

int tbs_plan_create(tbs_plan** out, int ndim, const int64_t grid[3], double dx, tbs_c128 k0,
                    int padding, int dtype, int batch, void* hip_stream) {
  if (!out) return fail(nullptr, TBS_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (ndim != 2 && ndim != 3) return fail(nullptr, TBS_ERR_INVALID, "ndim must be 2 or 3");
  if (!grid) return fail(nullptr, TBS_ERR_INVALID, "grid is NULL");
  if (!(dx > 0) || !is_fin(dx)) return fail(nullptr, TBS_ERR_INVALID, "dx must be > 0");
  if (!(k0.re > 0) || !(k0.im >= 0) || !is_fin(k0.re) || !is_fin(k0.im))
    return fail(nullptr, TBS_ERR_INVALID, "k0 needs Re k0 > 0 and Im k0 >= 0");
  if (padding < 1) return fail(nullptr, TBS_ERR_INVALID, "padding must be >= 1");
  if (dtype != TBS_C64 && dtype != TBS_C128) return fail(nullptr, TBS_ERR_INVALID, "bad dtype");
  if (batch < 1 || batch > 4096) return fail(nullptr, TBS_ERR_INVALID, "batch must be 1..4096");
  if (padding == 1) {
    // periodic plan: 2D, both sizes powers of two in [16, 4096]
    if (ndim != 2) return fail(nullptr, TBS_ERR_UNSUPPORTED, "periodic plans are 2D");
    for (int d = 0; d < 2; ++d) {
      const int64_t n = grid[d];
      if (n < 16 || n > 4096 || (n & (n - 1)) != 0)
        return fail(nullptr, TBS_ERR_UNSUPPORTED, "periodic grid sizes must be powers of two in [16, 4096]");
    }
  }
  tbs_plan* p = new (std::nothrow) tbs_plan();
  if (!p) return fail(nullptr, TBS_ERR_OOM, "host allocation failed");
  p->ndim = ndim;
  p->N[0] = grid[0];
  p->N[1] = grid[1];
  p->N[2] = ndim == 3 ? grid[2] : 1;
  p->periodic = padding == 1;
  for (int d = 0; d < ndim && p->periodic; ++d) p->M[d] = p->N[d];
  for (int d = 0; d < ndim && !p->periodic; ++d) {
    if (p->N[d] < 1 || p->N[d] > 2048) {
      delete p;
      return fail(nullptr, TBS_ERR_UNSUPPORTED, "grid sizes must be 1..2048");
    }
    int rc = tbs_padded_length(p->N[d], padding, &p->M[d]);
    if (rc) {
      delete p;
      return fail(nullptr, TBS_ERR_UNSUPPORTED, "no compiled FFT length for this grid size");
    }
  }
  p->dx = dx;
  p->k0 = zd{k0.re, k0.im};
  p->dtype = dtype;
  p->fp64 = dtype == TBS_C128;
  p->esz = p->fp64 ? 16 : 8;
  p->batch = batch;
  p->stream = (hipStream_t)hip_stream;
  p->P = p->N[0] * p->N[1] * p->N[2];
  p->cb = tbs::spectral_block((int)(ndim == 2 ? p->M[1] : p->M[2]), p->fp64);
  if (hipGetDevice(&p->device) != hipSuccess) {
    (void)hipGetLastError();
    delete p;
    return fail(nullptr, TBS_ERR_HIP, "no HIP device");
  }
  const size_t B = (size_t)batch;
  const size_t xe = B * p->M[0] * p->N[1] * p->N[2];
  p->X_bytes = xe * p->esz;
  int rc = dev_alloc(p, &p->X, p->X_bytes);
  p->xcur = p->X;
  if (!rc && ndim == 3) rc = dev_alloc(p, &p->Yb, B * p->M[0] * p->M[1] * p->N[2] * p->esz);
  if (!rc && !p->fp64 && !p->periodic) {
    p->kc_bytes = (size_t)((B * p->P * 4 + 7) / 8 * 8);
    rc = dev_alloc(p, &p->kc, p->kc_bytes);
  }
  if (!rc && p->periodic) rc = dev_alloc(p, &p->psi0, B * p->P * p->esz);
  if (!rc && p->periodic) rc = dev_alloc(p, (void**)&p->iflags, 2 * sizeof(int));
  p->ghat_n = (p->M[0] / 2 + 1) * (p->M[1] / 2 + 1) * (ndim == 3 ? p->M[2] / 2 + 1 : 1);
  if (!rc) rc = dev_alloc(p, &p->ghat, (size_t)p->ghat_n * p->esz);
  for (int d = 0; d < ndim && !rc; ++d) rc = upload_twiddles(p, (int)p->M[d], p->fp64, &p->tw[d]);
  if (rc) {
    g_create_err = p->err;
    tbs_plan_destroy(p);
    return rc;
  }
  *out = p;
  return TBS_OK;
}

int tbs_plan_info(const tbs_plan* p, int64_t padded[3], int64_t* bytes) {
  if (!p) return TBS_ERR_INVALID;
  if (padded) {
    padded[0] = p->M[0];
    padded[1] = p->M[1];
    padded[2] = p->ndim == 3 ? p->M[2] : 1;
  }
  if (bytes) *bytes = p->device_bytes;
  return TBS_OK;
}

int tbs_plan_set_stream(tbs_plan* p, void* s) {
  if (!p) return TBS_ERR_INVALID;
  p->stream = (hipStream_t)s;
  return TBS_OK;
}

int tbs_green_tabulate(tbs_plan* p) {
  if (!p) return TBS_ERR_INVALID;
  if (p->periodic) return fail(p, TBS_ERR_STATE, "periodic plans take tbs_green_periodic");
  const int64_t Mx = p->M[0], My = p->M[1], Mz = p->ndim == 3 ? p->M[2] : 1;
  const int64_t M3[3] = {Mx, My, Mz};
  void* W = nullptr;
  int rc = dev_alloc(p, &W, (size_t)(Mx * My * Mz) * 16);
  if (rc) return rc;
  void* tw64[3] = {nullptr, nullptr, nullptr};
  for (int d = 0; d < p->ndim && !rc; ++d) rc = upload_twiddles(p, (int)M3[d], true, &tw64[d]);
  auto cleanup = [&]() {
    dev_free(p, W, (size_t)(Mx * My * Mz) * 16);
    for (int d = 0; d < 3; ++d) dev_free(p, tw64[d], 0);
  };
  if (rc) {
    cleanup();
    return rc;
  }
  tbs_c128 w0;
  tbs_self_cell(p->ndim, tbs_c128{p->k0.re, p->k0.im}, p->dx, &w0);
  int e = tbs::launch_green_eval(W, p->ndim, M3, p->dx, p->k0.re, p->k0.im, w0.re, w0.im, p->stream);
  // x: contiguous rows
  if (!e) e = tbs::launch_row_fft_full((int)Mx, W, tw64[0], (int)(My * Mz), 0, p->stream);
  // y, then z: strided lines, 4 contiguous columns per block
  for (int ax = 1; ax < p->ndim && !e; ++ax) {
    const int nc = tbs::col_max_cols((int)M3[ax], true);
    tbs::ColArgs a{};
    a.sub = 1;
    a.in = W;
    a.out = W;
    a.tw = tw64[ax];
    a.op = tbs::COL_FULL;
    a.cb = nc;
    a.zcols = 0;
    a.zlim = 1;
    a.nrhs = 1;
    a.n0 = (int)(Mx / nc);
    a.in_s0 = a.out_s0 = nc;
    if (ax == 1) {
      a.n_in = a.n_out = (int)My;
      a.in_astride = a.out_astride = Mx;
      a.n1 = (int)Mz;
      a.in_s1 = a.out_s1 = My * Mx;
    } else {
      a.n_in = a.n_out = (int)Mz;
      a.in_astride = a.out_astride = Mx * My;
      a.n1 = (int)My;
      a.in_s1 = a.out_s1 = Mx;
    }
    a.xcd_remap = 0;
    e = tbs::launch_col_pass(true, (int)M3[ax], nc, a, p->stream);
  }
  if (!e) e = tbs::launch_green_fold(W, p->ghat, p->fp64, p->ndim, M3, p->stream);
  if (e) {
    cleanup();
    return hip_fail(p, (hipError_t)e, "green tabulation launch");
  }
  hipError_t he = hipStreamSynchronize(p->stream);
  cleanup();
  if (he != hipSuccess) return hip_fail(p, he, "green tabulation");
  p->green_ready = true;
  return TBS_OK;
}

int tbs_density_contrast(tbs_plan* p, const double* gamma) {
  if (!p) return TBS_ERR_INVALID;
  if (p->periodic) return fail(p, TBS_ERR_UNSUPPORTED, "the density term is built for padded plans");
  if (gamma && p->batch_refs > 0)
    return fail(p, TBS_ERR_STATE, "the plan belongs to a live batch (batches take no density term)");
  p->gamma = gamma;
  return TBS_OK;
}

int tbs_green_periodic(tbs_plan* p, double eps, const tbs_kspace_potential* vv) {
  if (!p) return TBS_ERR_INVALID;
  if (!p->periodic) return fail(p, TBS_ERR_STATE, "not a periodic plan (create it with padding 1)");
  if (!(eps >= 0) || !is_fin(eps)) return fail(p, TBS_ERR_INVALID, "eps must be finite and >= 0");
  if (vv && (!is_fin(vv->tau) || !is_fin(vv->eta) || !(vv->nu > 0) || !is_fin(vv->nu) ||
             !(vv->omega > 0) || !is_fin(vv->omega)))
    return fail(p, TBS_ERR_INVALID, "bad k-space potential parameters");
  if (vv && !p->ghat_vv) {
    int rc = dev_alloc(p, &p->ghat_vv, (size_t)p->ghat_n * p->esz);
    if (rc) return rc;
  } else if (!vv && p->ghat_vv) {
    TBS_HIP(p, hipStreamSynchronize(p->stream));
    dev_free(p, p->ghat_vv, (size_t)p->ghat_n * p->esz);
  }
  const double k2r = p->k0.re * p->k0.re - p->k0.im * p->k0.im;
  const double k2i = 2.0 * p->k0.re * p->k0.im;
  TBS_LAUNCH(p, tbs::launch_periodic_green(p->ghat, vv ? p->ghat_vv : nullptr, p->fp64, p->M[0],
                                           p->M[1], p->dx, k2r, k2i, eps, vv ? vv->tau : 0.0,
                                           vv ? vv->eta : 0.0, vv ? vv->nu : 1.0,
                                           vv ? vv->omega : 1.0, p->stream));
  p->eps = eps;
  p->green_ready = true;
  return TBS_OK;
}

int tbs_kspace_coefficients(double alpha0, double nu, double c, double omega,
                            tbs_kspace_potential* out) {
  if (!out || !(alpha0 >= 0) || !(nu > 0) || !(c > 0) || !(omega > 0) || !is_fin(alpha0) ||
      !is_fin(nu) || !is_fin(c) || !is_fin(omega))
    return TBS_ERR_INVALID;
  out->tau = -2.0 * alpha0 * std::pow(c, nu - 1.0);
  out->eta = 2.0 * alpha0 * std::pow(c, nu) * std::tan(tbs::kPi * nu / 2.0);
  out->nu = nu;
  out->omega = omega;
  return TBS_OK;
}

int tbs_abl_profile(int64_t n, double dx, double zeta, double mu_cells, double* out) {
  if (!out || n < 1 || !(dx > 0) || !(zeta >= 0) || !(mu_cells >= 0) || !is_fin(zeta) ||
      !is_fin(mu_cells))
    return TBS_ERR_INVALID;
  const double mu_cm = mu_cells * dx * 100.0;
  for (int64_t i = 0; i < n; ++i) {
    const double d_cm = (double)std::min(i, n - 1 - i) * dx * 100.0;
    out[i] = d_cm < mu_cm ? 1.0 / (1.0 + std::exp(-zeta * (d_cm - 0.5 * mu_cm))) : 1.0;
  }
  return TBS_OK;
}

int tbs_iterate(tbs_plan* p, const void* source, const void* V, const double* mask_x,
                const double* mask_y, int check_row, double tol, int max_iter, void* psi_out,
                int* iters_out, double* err_out, int flags) {
  if (!p) return TBS_ERR_INVALID;
  if (!p->periodic) return fail(p, TBS_ERR_STATE, "not a periodic plan (create it with padding 1)");
  if (!p->green_ready) return fail(p, TBS_ERR_STATE, "call tbs_green_periodic first");
  if (!source || !psi_out) return fail(p, TBS_ERR_INVALID, "NULL argument");
  if (max_iter < 1 || max_iter > 1000000) return fail(p, TBS_ERR_INVALID, "max_iter must be 1..1e6");
  if (check_row < 0 || check_row >= p->N[1]) return fail(p, TBS_ERR_INVALID, "check_row out of range");
  if (!(tol >= 0) || !is_fin(tol)) return fail(p, TBS_ERR_INVALID, "tol must be finite and >= 0");
  if (flags != TBS_ITER_PAPER && flags != TBS_ITER_CBS) return fail(p, TBS_ERR_INVALID, "bad flags");
  if (flags == TBS_ITER_CBS && (!V || !(p->eps > 0) || p->ghat_vv))
    return fail(p, TBS_ERR_INVALID, "the convergent series needs a potential, eps > 0 and no k-space table");
  if (psi_out == source || psi_out == V) return fail(p, TBS_ERR_INVALID, "psi_out aliases an input");
  int rc = ensure_doubles(p, &p->partials, &p->partials_cap, (size_t)2 * p->batch);
  if (!rc) rc = ensure_doubles(p, &p->ierrs, &p->ierrs_cap, (size_t)max_iter);
  if (rc) return rc;
  TBS_LAUNCH(p, tbs::launch_zero(p->iflags, (int64_t)(2 * sizeof(int)), p->stream));

  tbs::IterArgs a{};
  a.X = p->X;
  a.tw = p->tw[0];
  a.psi = psi_out;
  a.psi0 = p->psi0;
  a.src = source;
  a.V = V;
  a.mask_x = mask_x;
  a.mask_y = mask_y;
  a.partials = p->partials;
  a.done = nullptr;
  a.nx = (int)p->N[0];
  a.nrows = (int)p->N[1];
  a.nrhs = p->batch;
  a.check_row = check_row;
  a.cb = p->cb;
  a.cbs = flags == TBS_ITER_CBS ? 1 : 0;
  a.inv_eps = p->eps > 0 ? 1.0 / p->eps : 0.0;

  int nc = 0;
  tbs::ColArgs c = make_conv2d_args(p, false, &nc);
  c.op = tbs::COL_CONV_FULL;
  c.n_in = c.n_out = (int)p->N[1];
  const int Mx = (int)p->M[0], My = (int)p->M[1];

  // psi0 = G s (no absorbing layer on the first field)
  a.mode = tbs::ITER_SOURCE;
  TBS_LAUNCH(p, tbs::launch_iter_row(p->fp64, Mx, a, p->stream));
  TBS_LAUNCH(p, tbs::launch_iter_col(p->fp64, My, nc, c, nullptr, p->stream));
  a.mode = tbs::ITER_FIRST;
  TBS_LAUNCH(p, tbs::launch_iter_row(p->fp64, Mx, a, p->stream));

  a.mode = tbs::ITER_STEP;
  a.done = p->iflags;
  if (p->ghat_vv) c.ghat = p->ghat_vv;
  int dflags[2] = {0, 0};
  const int chunk = 8;
  for (int it = 1; it <= max_iter;) {
    const int end = std::min(max_iter, it + chunk - 1);
    for (; it <= end; ++it) {
      TBS_LAUNCH(p, tbs::launch_iter_col(p->fp64, My, nc, c, p->iflags, p->stream));
      TBS_LAUNCH(p, tbs::launch_iter_row(p->fp64, Mx, a, p->stream));
      TBS_LAUNCH(p, tbs::launch_iter_finish(p->partials, p->batch, it, tol, p->ierrs, p->iflags,
                                            p->iflags + 1, p->stream));
    }
    TBS_HIP(p, hipMemcpyAsync(dflags, p->iflags, sizeof(dflags), hipMemcpyDeviceToHost, p->stream));
    TBS_HIP(p, hipStreamSynchronize(p->stream));
    if (dflags[0]) break;
  }
  const int n = dflags[1];
  if (iters_out) *iters_out = n;
  std::vector<double> errs((size_t)std::max(n, 1), 0.0);
  if (n > 0)
    TBS_HIP(p, hipMemcpy(errs.data(), p->ierrs, (size_t)n * sizeof(double), hipMemcpyDeviceToHost));
  if (err_out && n > 0) std::memcpy(err_out, errs.data(), (size_t)n * sizeof(double));
  for (int i = 0; i < n; ++i)
    if (!is_fin(errs[(size_t)i])) return fail(p, TBS_WARN_NONFINITE, "non-finite iteration error");
  if (!dflags[0]) return fail(p, TBS_WARN_NOT_CONVERGED, "tolerance not reached within max_iter");
  return TBS_OK;
}

int tbs_green_import(tbs_plan* p, const tbs_c128* full) {
  if (!p || !full) return fail(p, TBS_ERR_INVALID, "NULL argument");
  const int64_t Mx = p->M[0], My = p->M[1], Mz = p->ndim == 3 ? p->M[2] : 1;
  const int64_t hx = Mx / 2 + 1, hy = My / 2 + 1, hz = Mz / 2 + 1;
  const double sc = 1.0 / ((double)Mx * (double)My * (double)Mz);
  std::vector<double> buf(2 * (size_t)p->ghat_n);
  for (int64_t fx = 0; fx < hx; ++fx)
    for (int64_t fy = 0; fy < hy; ++fy)
      for (int64_t fz = 0; fz < hz; ++fz) {
        const tbs_c128 v = full[(fz * My + fy) * Mx + fx];
        const size_t i = (size_t)((fx * hy + fy) * hz + fz);
        buf[2 * i] = v.re * sc;
        buf[2 * i + 1] = v.im * sc;
      }
  if (p->fp64) {
    TBS_HIP(p, hipMemcpy(p->ghat, buf.data(), buf.size() * 8, hipMemcpyHostToDevice));
  } else {
    std::vector<float> f(buf.size());
    for (size_t i = 0; i < buf.size(); ++i) f[i] = (float)buf[i];
    TBS_HIP(p, hipMemcpy(p->ghat, f.data(), f.size() * 4, hipMemcpyHostToDevice));
  }
  p->green_ready = true;
  return TBS_OK;
}

int tbs_green_export(const tbs_plan* pc, tbs_c128* out) {
  tbs_plan* p = const_cast<tbs_plan*>(pc);
  if (!p || !out) return fail(p, TBS_ERR_INVALID, "NULL argument");
  if (!p->green_ready) return fail(p, TBS_ERR_STATE, "no spectrum tabulated");
  TBS_HIP(p, hipStreamSynchronize(p->stream));
  if (p->fp64) {
    TBS_HIP(p, hipMemcpy(out, p->ghat, (size_t)p->ghat_n * 16, hipMemcpyDeviceToHost));
  } else {
    std::vector<float> f(2 * (size_t)p->ghat_n);
    TBS_HIP(p, hipMemcpy(f.data(), p->ghat, f.size() * 4, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < p->ghat_n; ++i) out[i] = tbs_c128{f[2 * i], f[2 * i + 1]};
  }
  return TBS_OK;
}

int tbs_potential(tbs_plan* p, const double* c, double omega, double c0, double alpha0, double y,
                  double eps, void* V, void* dVdc) {
  if (!p || !c) return fail(p, TBS_ERR_INVALID, "NULL argument");
  if (!(omega > 0) || !(c0 > 0) || !(alpha0 >= 0) || !(eps >= 0) || !is_fin(y))
    return fail(p, TBS_ERR_INVALID, "bad medium parameters");
  const double a = alpha0 * std::pow(omega, y);
  const double disp = (std::fabs(y - 1.0) < 1e-12) ? 0.0 : std::tan(tbs::kPi * y / 2.0);
  const double kr = omega / c0 + a * disp, ki = a;
  const double k0r = kr * kr - ki * ki, k0i = 2.0 * kr * ki + eps;
  TBS_LAUNCH(p, tbs::launch_potential(c, V, dVdc, p->fp64, p->P, omega, a, disp, k0r, k0i,
                                      p->stream));
  return TBS_OK;
}

int tbs_solve(tbs_plan* p, const void* source, const void* V, int nterms, void* p_out,
              double* residual_out) {
  int rc = check_plan_ready(p);
  if (rc) return rc;
  if (!source || !p_out) return fail(p, TBS_ERR_INVALID, "source and p_out are required");
  if (nterms < 1 || nterms > 100000) return fail(p, TBS_ERR_INVALID, "nterms must be >= 1");
  if (p_out == source || p_out == V) return fail(p, TBS_ERR_INVALID, "p_out aliases an input");
  rc = forward_series(p, source, V, nterms, p_out, nullptr);
  if (rc) return rc;
  if (residual_out) return check_residuals(p, residual_out, nterms);
  return TBS_OK;
}

int tbs_solve_noalloc(tbs_plan* p, const void* source, const void* V, int nterms, void* p_out,
                      double* residual_out) {
  int rc = check_plan_ready(p);
  if (rc) return rc;
  if (!source || !p_out) return fail(p, TBS_ERR_INVALID, "source and p_out are required");
  if (nterms < 1 || nterms > 100000) return fail(p, TBS_ERR_INVALID, "nterms must be >= 1");
  if (p_out == source || p_out == V) return fail(p, TBS_ERR_INVALID, "p_out aliases an input");
  if (p->gamma)
    return fail(p, TBS_ERR_UNSUPPORTED, "density-contrast plans keep a spatial term buffer: use tbs_solve");
  // workspace layout in the scratch array: X | 3D y intermediate | Kahan
  // compensation | norm partials | residuals (each 256-byte aligned); every
  // region is written before it is read, so nothing needs clearing
  const size_t B = (size_t)p->batch;
  const size_t L = (size_t)nterms;
  const size_t x_bytes = align256(p->X_bytes);
  const size_t y_bytes = p->ndim == 3 ? align256(B * p->M[0] * p->M[1] * p->N[2] * p->esz) : 0;
  const size_t c_bytes = p->kc ? align256(p->kc_bytes) : 0;
  const size_t part_n = (size_t)2 * B * row_blocks(p) * L;
  const size_t part_bytes = align256(part_n * sizeof(double));
  const size_t res_bytes = align256(B * L * sizeof(double));
  const size_t need = x_bytes + y_bytes + c_bytes + part_bytes + res_bytes;
  if (need > TBS_SCRATCH_BYTES)
    return fail(p, TBS_ERR_UNSUPPORTED,
                "tbs_solve_noalloc: the workspace of " + std::to_string(need) +
                    " bytes exceeds the static scratch of " + std::to_string(TBS_SCRATCH_BYTES) +
                    " bytes (use tbs_solve)");
  void* base = nullptr;
  rc = scratch_address(p, &base);
  if (rc) return rc;
  char* w = (char*)base;
  // run the plan's series on the scratch regions, then restore its own buffers
  void* const sv_X = p->X;
  void* const sv_xcur = p->xcur;
  void* const sv_Yb = p->Yb;
  void* const sv_kc = p->kc;
  double* const sv_part = p->partials;
  const size_t sv_part_cap = p->partials_cap;
  double* const sv_res = p->resid;
  const size_t sv_res_cap = p->resid_cap;
  const bool sv_prof = p->prof;
  p->X = p->xcur = w;
  if (y_bytes) p->Yb = w + x_bytes;
  if (c_bytes) p->kc = w + x_bytes + y_bytes;
  p->partials = (double*)(w + x_bytes + y_bytes + c_bytes);
  p->partials_cap = part_n;
  p->resid = (double*)(w + x_bytes + y_bytes + c_bytes + part_bytes);
  p->resid_cap = B * L;
  p->prof = false;  // profiling events are created on demand
  rc = forward_series(p, source, V, nterms, p_out, nullptr);
  if (!rc && residual_out) rc = check_residuals(p, residual_out, nterms);
  p->X = sv_X;
  p->xcur = sv_xcur;
  p->Yb = sv_Yb;
  p->kc = sv_kc;
  p->partials = sv_part;
  p->partials_cap = sv_part_cap;
  p->resid = sv_res;
  p->resid_cap = sv_res_cap;
  p->prof = sv_prof;
  return rc;
}

int tbs_harmonic_source(tbs_plan* p, const void* p1, const double* c, double omega, double rho,
                        double BA, void* S2) {
  if (!p || !p1 || !c || !S2) return fail(p, TBS_ERR_INVALID, "NULL argument");
  if (!(omega > 0) || !(rho > 0) || !is_fin(BA)) return fail(p, TBS_ERR_INVALID, "bad parameters");
  const double coef = -0.5 * (1.0 + 0.5 * BA) / rho * (2.0 * omega) * (2.0 * omega);
  TBS_LAUNCH(p, tbs::launch_harmonic_source(p1, c, S2, p->fp64, p->P, p->batch, coef, p->stream));
  return TBS_OK;
}

int tbs_harmonic_source_n(tbs_plan* p, int n, const void* const* fields, const double* c,
                          double omega, double rho, double BA, void* S) {
  if (!p || !fields || !c || !S) return fail(p, TBS_ERR_INVALID, "NULL argument");
  if (n < 2 || n > TBS_HARMONIC_MAX) return fail(p, TBS_ERR_INVALID, "harmonic order must be 2..9");
  for (int a = 0; a < n - 1; ++a)
    if (!fields[a]) return fail(p, TBS_ERR_INVALID, "NULL lower-harmonic field");
  if (!(omega > 0) || !(rho > 0) || !is_fin(BA)) return fail(p, TBS_ERR_INVALID, "bad parameters");
  const double nw = (double)n * omega;
  const double coef = -0.5 * (1.0 + 0.5 * BA) / rho * nw * nw;
  TBS_LAUNCH(p, tbs::launch_harmonic_source_n(n, fields, nullptr, c, S, p->fp64, p->P, p->batch, coef,
                                              1.0, p->stream));
  return TBS_OK;
}

int tbs_harmonic_source_scaled(tbs_plan* p, int n, const void* const* fields, const int* field_exp,
                               const double* c, double omega, double rho, double BA, void* S,
                               int* exp_out) {
  if (!p || !fields || !field_exp || !c || !S || !exp_out) return fail(p, TBS_ERR_INVALID, "NULL argument");
  if (n < 2 || n > TBS_HARMONIC_MAX) return fail(p, TBS_ERR_INVALID, "harmonic order must be 2..9");
  double unscale[TBS_HARMONIC_MAX - 1];
  for (int a = 0; a < n - 1; ++a) {
    if (!fields[a]) return fail(p, TBS_ERR_INVALID, "NULL lower-harmonic field");
    if (field_exp[a] < -900 || field_exp[a] > 900) return fail(p, TBS_ERR_INVALID, "field exponent out of range");
    unscale[a] = std::ldexp(1.0, -field_exp[a]);
  }
  if (!(omega > 0) || !(rho > 0) || !is_fin(BA)) return fail(p, TBS_ERR_INVALID, "bad parameters");
  const double nw = (double)n * omega;
  const double coef = -0.5 * (1.0 + 0.5 * BA) / rho * nw * nw;
  int rc = ensure_doubles(p, &p->jpart, &p->jpart_cap, (size_t)tbs::kHarmonicMaxSlots);
  if (rc) return rc;
  TBS_LAUNCH(p, tbs::launch_harmonic_source_n_max(n, fields, unscale, c, p->fp64, p->P, p->batch, coef,
                                                  p->jpart, p->stream));
  double mx = 0.0;
  TBS_HIP(p, hipMemcpyAsync(&mx, p->jpart + (tbs::kHarmonicMaxSlots - 1), sizeof(double),
                            hipMemcpyDeviceToHost, p->stream));
  TBS_HIP(p, hipStreamSynchronize(p->stream));
  if (!is_fin(mx)) return fail(p, TBS_ERR_INVALID, "non-finite harmonic source (non-finite fields?)");
  // 2^e brings the largest component into [1, 2)
  const int e = mx > 0.0 ? -std::ilogb(mx) : 0;
  TBS_LAUNCH(p, tbs::launch_harmonic_source_n(n, fields, unscale, c, S, p->fp64, p->P, p->batch, coef,
                                              std::ldexp(1.0, e), p->stream));
  *exp_out = e;
  return TBS_OK;
}

int tbs_adjoint(tbs_plan* p, const void* source, const void* V, int L, const void* q, void* grad,
                double* residual_out, int flags) {
  int rc = check_plan_ready(p);
  if (rc) return rc;
  if (p->gamma) return fail(p, TBS_ERR_UNSUPPORTED, "no adjoint with a density contrast");
  if (L < 1 || L > 100000) return fail(p, TBS_ERR_INVALID, "nterms must be >= 1");
  if (flags == TBS_ADJ_SERIES_ONLY) {
    // the adjoint field sum_{m<L} (G^H conj(V))^m G^H q: the forward passes
    // with conj(G^) and conj(V)
    if (!q || !grad) return fail(p, TBS_ERR_INVALID, "NULL argument");
    if (grad == q || grad == V) return fail(p, TBS_ERR_INVALID, "grad_out aliases an input");
    rc = forward_series(p, q, V, L, grad, nullptr, true);
    if (rc) return rc;
    if (residual_out) return check_residuals(p, residual_out, L);
    return TBS_OK;
  }
  if (!source || !V || !q || !grad) return fail(p, TBS_ERR_INVALID, "NULL argument");
  if (flags != TBS_ADJ_STORE && flags != TBS_ADJ_RECOMPUTE)
    return fail(p, TBS_ERR_INVALID, "bad flags");
  const size_t slot = (size_t)p->batch * p->P * p->esz;
  TBS_LAUNCH(p, tbs::launch_zero(grad, (int64_t)slot, p->stream));
  if (L == 1) {
    if (residual_out) {
      // forward residuals still requested
      void* tmp = nullptr;
      rc = dev_alloc(p, &tmp, slot);
      if (rc) return rc;
      rc = forward_series(p, source, V, 1, tmp, nullptr);
      int r2 = rc ? rc : check_residuals(p, residual_out, 1);
      (void)hipStreamSynchronize(p->stream);
      dev_free(p, tmp, slot);
      return r2;
    }
    return TBS_OK;
  }
  if (flags == TBS_ADJ_RECOMPUTE) return adjoint_recompute(p, source, V, L, q, grad, residual_out);
  // Forward pass keeping the partial sums P_1..P_{L-1} (the final p is not needed).
  // L-1 partial-sum slots and one more for the running sum
  const size_t need = slot * (size_t)(L - 1);
  if (p->pstore_bytes < need + slot) {
    dev_free(p, p->pstore, p->pstore_bytes);
    p->pstore_bytes = 0;
    rc = dev_alloc(p, &p->pstore, need + slot);
    if (rc) return rc;
    p->pstore_bytes = need + slot;
  }
  void* pacc = (char*)p->pstore + need;  // running sum buffer
  (void)flags;
  rc = forward_series(p, source, V, L, pacc, p->pstore);
  if (rc) return rc;
  if (residual_out) {
    rc = check_residuals(p, residual_out, L);
    if (rc < 0) return rc;
  }
  // Adjoint series: w_0 = G^H q; row pass m pairs w_m with P_{L-1-m} and
  // forms conj(V) w_m for the next term, m = 0..L-2.
  const int nblk = row_blocks(p);
  rc = run_row(p, tbs::ROW_IN_SOURCE, tbs::ACC_NONE, 1, true, q, nullptr, nullptr, nullptr,
               nullptr, nullptr, nullptr);
  if (rc) return rc;
  rc = run_cols(p, true);
  if (rc) return rc;
  (void)nblk;
  for (int m = 0; m <= L - 2; ++m) {
    const void* pair = (const char*)p->pstore + (size_t)(L - 2 - m) * slot;  // P_{L-1-m}
    const bool more = m < L - 2;
    rc = run_row(p, tbs::ROW_IN_SPECTRAL, tbs::ACC_PAIR, more ? 1 : 0, true, nullptr, V, nullptr,
                 nullptr, pair, grad, p->partials);
    if (rc) return rc;
    if (more) {
      rc = run_cols(p, true);
      if (rc) return rc;
    }
  }
  return TBS_OK;
}

int tbs_misfit(tbs_plan* p, const void* pf, const int64_t* rec, int nrec, const void* pobs,
               void* q, double* J) {
  if (!p || !pf || !rec || !pobs || !q || !J || nrec < 1)
    return fail(p, TBS_ERR_INVALID, "bad misfit arguments");
  const size_t slot = (size_t)p->batch * p->P * p->esz;
  int rc = ensure_doubles(p, &p->jpart, &p->jpart_cap, (size_t)nrec * p->batch);
  if (rc) return rc;
  TBS_LAUNCH(p, tbs::launch_zero(q, (int64_t)slot, p->stream));
  TBS_LAUNCH(p, tbs::launch_misfit(pf, rec, pobs, q, p->jpart, p->fp64, p->P, nrec, p->batch,
                                   p->stream));
  TBS_LAUNCH(p, tbs::launch_sum_half(p->jpart, nrec * p->batch, J, p->stream));
  return TBS_OK;
}

int tbs_speed_gradient(tbs_plan* p, const void* g, const void* dVdc, double* grad_c,
                       int accumulate) {
  if (!p || !g || !dVdc || !grad_c) return fail(p, TBS_ERR_INVALID, "NULL argument");
  TBS_LAUNCH(p, tbs::launch_grad_assemble(g, p->batch, dVdc, grad_c, p->fp64, p->P, accumulate,
                                          p->stream));
  return TBS_OK;
}

int tbs_plan_autotune(tbs_plan* p, int* row_nr_out, int* conv_nc_out) {
  if (!p) return TBS_ERR_INVALID;
  if (p->periodic) return fail(p, TBS_ERR_STATE, "periodic plans are not tuned");
  if (!p->green_ready) return fail(p, TBS_ERR_STATE, "tabulate the spectrum before tuning");
  if (p->batch_refs > 0)
    return fail(p, TBS_ERR_STATE, "the plan belongs to a live batch (tune before tbs_batch_create)");
  if (p->ndim == 2) {
    const std::string key = "plan " + device_tag(p->device) + " " + (p->fp64 ? "c128" : "c64") + " N" +
                            std::to_string(p->N[0]) + "x" + std::to_string(p->N[1]) + " M" +
                            std::to_string(p->M[0]) + "x" + std::to_string(p->M[1]) + " B" +
                            std::to_string(p->batch);
    bool hit = false;
    {
      std::vector<int> v;
      int cr[8], cc[8];
      const int nrn = tbs::row_nr_candidates((int)p->M[0], p->fp64, cr);
      const int ncn = tbs::conv_nc_candidates((int)p->M[1], p->fp64, p->cb, cc);
      if (tune_lookup(key, &v) && v.size() == 2 && in_list(v[0], cr, nrn) && in_list(v[1], cc, ncn)) {
        p->row_nr = v[0];
        p->conv_nc = v[1];
        hit = true;
      }
    }
    if (!hit) {
      const size_t slot = (size_t)p->batch * p->P * p->esz;
      void* pacc = nullptr;
      void* vz = nullptr;
      int rc = dev_alloc(p, &pacc, slot);
      if (!rc) rc = dev_alloc(p, &vz, (size_t)p->P * p->esz);
      const size_t per_term = (size_t)2 * p->batch * (size_t)p->N[1];  // >= 2 * batch * row blocks
      if (!rc) rc = ensure_doubles(p, &p->partials, &p->partials_cap, per_term);
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (!rc && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        rc = hip_fail(p, hipErrorOutOfMemory, "events");
      if (!rc) {
        (void)tbs::launch_zero(pacc, (int64_t)slot, p->stream);
        (void)tbs::launch_zero(vz, (int64_t)(p->P * p->esz), p->stream);
        (void)tbs::launch_zero(p->X, (int64_t)p->X_bytes, p->stream);
        if (p->kc) (void)tbs::launch_zero(p->kc, (int64_t)p->kc_bytes, p->stream);
      }
      auto timeit = [&](auto&& fn) -> double {
        for (int w = 0; w < 2; ++w) fn();
        (void)hipEventRecord(e0, p->stream);
        for (int r = 0; r < 5; ++r) fn();
        (void)hipEventRecord(e1, p->stream);
        (void)hipEventSynchronize(e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        return ms / 5.0;
      };
      int cand[8];
      if (!rc) {
        const int nrn = tbs::row_nr_candidates((int)p->M[0], p->fp64, cand);
        double best = 1e30;
        int pick = cand[0];
        for (int i = 0; i < nrn; ++i) {
          p->row_nr = cand[i];
          const tbs::RowArgs a = make_row_args(p, tbs::ROW_IN_SPECTRAL, tbs::ACC_ADD, 1, false, nullptr,
                                               vz, pacc, nullptr, nullptr, nullptr, p->partials);
          const double t = timeit([&] {
            (void)tbs::launch_row_pass(p->fp64, (int)p->M[0], a, row_blocks(p), p->row_nr, p->stream);
          });
          if (t < best) {
            best = t;
            pick = cand[i];
          }
        }
        p->row_nr = pick;
        const int ncn = tbs::conv_nc_candidates((int)p->M[1], p->fp64, p->cb, cand);
        best = 1e30;
        pick = cand[0];
        for (int i = 0; i < ncn; ++i) {
          p->conv_nc = cand[i];
          int nc = 0;
          const tbs::ColArgs c = make_conv2d_args(p, false, &nc);
          const double t = timeit([&] {
            (void)tbs::launch_col_pass(p->fp64, (int)p->M[1], nc, c, p->stream);
          });
          if (t < best) {
            best = t;
            pick = cand[i];
          }
        }
        p->conv_nc = pick;
        hipError_t he = hipStreamSynchronize(p->stream);
        if (he != hipSuccess) rc = hip_fail(p, he, "autotune");
      }
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
      dev_free(p, pacc, slot);
      dev_free(p, vz, (size_t)p->P * p->esz);
      if (rc) {
        p->row_nr = 0;
        p->conv_nc = 0;
        return rc;
      }
      tune_store(key, {p->row_nr, p->conv_nc});
    }
  } else {
    // 3D: z lines per block of the z convolution (its y passes and the x row
    // pass have one compiled shape at these lengths)
    const std::string key = "plan3 " + device_tag(p->device) + " " + (p->fp64 ? "c128" : "c64") + " N" +
                            std::to_string(p->N[0]) + "x" + std::to_string(p->N[1]) + "x" +
                            std::to_string(p->N[2]) + " M" + std::to_string(p->M[0]) + "x" +
                            std::to_string(p->M[1]) + "x" + std::to_string(p->M[2]) + " B" +
                            std::to_string(p->batch);
    int cand[8];
    const int n = tbs::conv_nc_candidates((int)p->M[2], p->fp64, p->cb, cand);
    std::vector<int> v;
    if (tune_lookup(key, &v) && v.size() == 1 && in_list(v[0], cand, n)) {
      p->conv_nc = v[0];
    } else if (n > 1) {
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        (void)hipGetLastError();
        if (e0) (void)hipEventDestroy(e0);
        return hip_fail(p, hipErrorOutOfMemory, "events");
      }
      double best = 1e30;
      int pick = cand[0];
      int rc = TBS_OK;
      for (int i = 0; i < n && !rc; ++i) {
        p->conv_nc = cand[i];
        for (int w = 0; w < 2 && !rc; ++w) rc = run_cols(p, false);
        (void)hipEventRecord(e0, p->stream);
        for (int r = 0; r < 3 && !rc; ++r) rc = run_cols(p, false);
        (void)hipEventRecord(e1, p->stream);
        if (rc || hipEventSynchronize(e1) != hipSuccess) break;
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ms < best) {
          best = ms;
          pick = cand[i];
        }
      }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      p->conv_nc = rc ? 0 : pick;
      if (rc) return rc;
      tune_store(key, {pick});
    }
  }
  if (row_nr_out) *row_nr_out = p->row_nr ? p->row_nr : tbs::row_rows_per_block((int)p->M[0], p->fp64);
  if (conv_nc_out) {
    int nc = 0;
    if (p->ndim == 2) (void)make_conv2d_args(p, false, &nc);
    else nc = p->conv_nc ? p->conv_nc : p->cb;
    *conv_nc_out = nc;
  }
  return TBS_OK;
}

int tbs_profile_enable(tbs_plan* p, int enable) {
  if (!p) return TBS_ERR_INVALID;
  TBS_HIP(p, hipStreamSynchronize(p->stream));
  p->prof = enable != 0;
  p->ev_used = 0;
  p->ev_marks.clear();
  return TBS_OK;
}

int tbs_profile_read(tbs_plan* p, double* ms, int64_t* cnt) {
  if (!p || !ms || !cnt) return fail(p, TBS_ERR_INVALID, "NULL argument");
  TBS_HIP(p, hipStreamSynchronize(p->stream));
  for (int k = 0; k < PK_N; ++k) {
    ms[k] = 0.0;
    cnt[k] = 0;
  }
  for (const auto& m : p->ev_marks) {
    float t = 0.0f;
    TBS_HIP(p, hipEventElapsedTime(&t, p->ev_pool[m.second], p->ev_pool[m.second + 1]));
    ms[m.first] += t;
    cnt[m.first] += 1;
  }
  p->ev_used = 0;
  p->ev_marks.clear();
  return TBS_OK;
}

int tbs_batch_create(tbs_batch** out, tbs_plan* const* plans, int nplans) {
  if (!out) return TBS_ERR_INVALID;
  *out = nullptr;
  if (!plans || nplans < 1) return fail(nullptr, TBS_ERR_INVALID, "empty batch");
  tbs_batch* b = new (std::nothrow) tbs_batch();
  if (!b) return fail(nullptr, TBS_ERR_OOM, "host allocation failed");
  for (int i = 0; i < nplans; ++i) {
    tbs_plan* p = plans[i];
    if (!p || p->ndim != 2 || p->periodic || p->gamma || !p->green_ready || p->fp64 != plans[0]->fp64) {
      delete b;
      return fail(nullptr, TBS_ERR_INVALID,
                  "batch plans must be 2D, tabulated and of one dtype");
    }
    b->plans.push_back(p);
  }
  b->fp64 = plans[0]->fp64;
  // A graph can only be recorded on a created stream (not the null stream):
  // the batch owns one (default priority) and joins the caller's stream with
  // events around every replay.
  if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    tbs_batch_destroy(b);
    return fail(nullptr, TBS_ERR_HIP, "batch stream/events");
  }
  // launch chains: TBS_BATCH_CHAINS (1 .. 4), default 3
  b->chains = TBS_BATCH_CHAINS_DEFAULT;
  if (const char* env = std::getenv("TBS_BATCH_CHAINS")) b->chains = std::atoi(env);
  b->chains = std::max(1, std::min(kMaxChains, b->chains));
  // streams for every chain count tbs_batch_autotune may choose
  bool ok = hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming) == hipSuccess;
  for (int c = 1; ok && c < kMaxChains; ++c)
    ok = hipStreamCreateWithFlags(&b->cstream[c], hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&b->ev_join[c], hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    tbs_batch_destroy(b);
    return fail(nullptr, TBS_ERR_HIP, "batch chain streams/events");
  }
  // one set of whole plans: the chains balanced by work (points x
  // right-hand sides), largest plan first to the lightest chain
  b->chain_of.assign(nplans, 0);
  {
    std::vector<int> order(nplans);
    for (int i = 0; i < nplans; ++i) order[i] = i;
    auto work = [&](int i) { return (double)b->plans[i]->M[0] * b->plans[i]->M[1] * b->plans[i]->batch; };
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work(x) > work(y); });
    double w[kMaxChains] = {0.0, 0.0, 0.0, 0.0};
    for (int i : order) {
      const int c = (int)(std::min_element(w, w + b->chains) - w);
      b->chain_of[i] = c;
      w[c] += work(i);
    }
  }
  int grc = batch_group(b);
  if (grc) {
    tbs_batch_destroy(b);
    return fail(nullptr, grc, "batch tables");
  }
  for (tbs_plan* p : b->plans) p->batch_refs += 1;
  b->counted = true;
  *out = b;
  return TBS_OK;
}

int tbs_batch_solve(tbs_batch* b, const void* const* sources, const void* const* potentials,
                    int L, void* const* p_outs, double* residual_out) {
  if (!b) return TBS_ERR_INVALID;
  if (!sources || !potentials || !p_outs) return bfail(b, TBS_ERR_INVALID, "NULL pointer array");
  if (L < 1 || L > 100000) return bfail(b, TBS_ERR_INVALID, "nterms must be >= 1");
  const int np = (int)b->plans.size();
  std::vector<const void*> key;
  for (int i = 0; i < np; ++i) {
    if (!sources[i] || !potentials[i] || !p_outs[i])
      return bfail(b, TBS_ERR_INVALID, "batch solves need source, potential and output per plan");
    key.push_back(sources[i]);
    key.push_back(potentials[i]);
    key.push_back(p_outs[i]);
  }
  // plan-owned buffers and block shapes the recorded launches hold
  for (tbs_plan* p : b->plans) {
    key.push_back(p->ghat);
    key.push_back(p->partials);
    key.push_back(p->resid);
    key.push_back(p->X);
    key.push_back(p->kc);
    key.push_back((const void*)(intptr_t)p->row_nr);
    key.push_back((const void*)(intptr_t)p->conv_nc);
  }
  const bool ready = b->tables_ready && key == b->key && L == b->key_L;
  if (!ready) {
    // a previous solve may still read the descriptor tables
    if (!batch_sync(b)) return bfail(b, TBS_ERR_HIP, "batch: previous solve failed");
    batch_drop_graph(b);
    // per-plan scratch for L terms, then the descriptor tables
    for (tbs_plan* p : b->plans) {
      const size_t per_term = (size_t)2 * p->batch * row_blocks(p);
      if (ensure_doubles(p, &p->partials, &p->partials_cap, per_term * (size_t)L) ||
          ensure_doubles(p, &p->resid, &p->resid_cap, (size_t)p->batch * L))
        return bfail(b, TBS_ERR_OOM, p->err);
    }
    const int nt = (int)b->tiles.size();
    std::vector<tbs::RowArgs> rows((size_t)(L + 1) * nt);
    std::vector<tbs::ColArgs> cols((size_t)nt);
    for (int t = 0; t < nt; ++t) {
      const int i = b->tiles[t].plan;
      for (int n = 0; n <= L; ++n)
        rows[(size_t)n * nt + b->rpos[t]] = tile_row_args(b, t, n, L, sources[i], potentials[i], p_outs[i]);
      cols[b->cpos[t]] = tile_col_args(b, t);
    }
    const size_t rb = rows.size() * sizeof(tbs::RowArgs);
    if (b->d_row_bytes < rb) {
      if (b->d_row) (void)hipFree(b->d_row);
      b->d_row = nullptr;
      b->d_row_bytes = 0;
      if (hipMalloc(&b->d_row, rb) != hipSuccess) {
        (void)hipGetLastError();
        return bfail(b, TBS_ERR_OOM, "batch descriptor table");
      }
      b->d_row_bytes = rb;
    }
    if (!b->d_col && hipMalloc(&b->d_col, cols.size() * sizeof(tbs::ColArgs)) != hipSuccess) {
      (void)hipGetLastError();
      b->d_col = nullptr;
      return bfail(b, TBS_ERR_OOM, "batch descriptor table");
    }
    if (hipMemcpy(b->d_row, rows.data(), rb, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->d_col, cols.data(), cols.size() * sizeof(tbs::ColArgs), hipMemcpyHostToDevice) !=
            hipSuccess)
      return bfail(b, TBS_ERR_HIP, "descriptor upload failed");
    b->key = key;
    b->key_L = L;
    b->tables_ready = true;
  }
  const hipStream_t caller = b->plans[0]->stream;
  if (b->prof) {
    // profiled: the launches go straight to the batch stream (no graph)
    hipError_t e = hipEventRecord(b->ev_in, caller);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, b->ev_in, 0);
    if (e != hipSuccess) return bfail(b, TBS_ERR_HIP, std::string("batch stream join: ") + hipGetErrorString(e));
    int rc = batch_enqueue(b, L);
    if (rc) return rc;
  } else if (!b->exec) {
    // record the sequence as a graph
    hipGraph_t graph = nullptr;
    if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      (void)hipGetLastError();
      return bfail(b, TBS_ERR_HIP, "graph capture could not start");
    }
    int rc = batch_enqueue(b, L);
    hipError_t e = hipStreamEndCapture(b->stream, &graph);
    if (rc) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (e != hipSuccess) return bfail(b, TBS_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      b->exec = nullptr;
      return bfail(b, TBS_ERR_HIP, std::string("graph instantiation: ") + hipGetErrorString(e));
    }
  }
  // caller's stream -> batch stream -> caller's stream
  hipError_t e = hipSuccess;
  if (!b->prof) {
    e = hipEventRecord(b->ev_in, caller);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, b->ev_in, 0);
    if (e == hipSuccess) e = hipGraphLaunch(b->exec, b->stream);
  }
  if (e == hipSuccess) e = hipEventRecord(b->ev_out, b->stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(caller, b->ev_out, 0);
  if (e != hipSuccess) return bfail(b, TBS_ERR_HIP, std::string("graph launch: ") + hipGetErrorString(e));
  if (!residual_out) return TBS_OK;
  e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return bfail(b, TBS_ERR_HIP, std::string("batch: ") + hipGetErrorString(e));
  int warn = TBS_OK;
  size_t off = 0;
  for (tbs_plan* p : b->plans) {
    int rc = check_residuals(p, residual_out + off, L);
    if (rc < 0) return bfail(b, rc, p->err);
    if (rc > 0 && warn == TBS_OK) {
      warn = rc;
      b->err = p->err;
    }
    off += (size_t)p->batch * L;
  }
  return warn;
}

int tbs_batch_autotune(tbs_batch* b, const void* const* sources, const void* const* potentials,
                       void* const* p_outs) {
  if (!b) return TBS_ERR_INVALID;
  if (!sources || !potentials || !p_outs) return bfail(b, TBS_ERR_INVALID, "NULL pointer array");
  const int np = (int)b->plans.size();
  for (int i = 0; i < np; ++i)
    if (!sources[i] || !potentials[i] || !p_outs[i])
      return bfail(b, TBS_ERR_INVALID, "batch tuning needs source, potential and output per plan");
  if (!batch_sync(b)) return bfail(b, TBS_ERR_HIP, "batch: previous solve failed");
  batch_drop_graph(b);
  const hipStream_t s = b->plans[0]->stream;
  for (tbs_plan* p : b->plans) {
    // norm partials of two row passes (a middle term) for any block shape
    // (at most one row per block)
    if (ensure_doubles(p, &p->partials, &p->partials_cap, (size_t)4 * p->batch * p->N[1]))
      return bfail(b, TBS_ERR_OOM, p->err);
  }
  // the tiles and sets the solves will run (the block shapes do not change them)
  int grc0 = batch_group(b);
  if (grc0) return bfail(b, grc0, "batch tables");
  const int nt = (int)b->tiles.size();
  const std::string tag = device_tag(b->plans[0]->device) + (b->fp64 ? " c128" : " c64");
  const std::string sched = b->nsets > 1 || b->tile_rhs
                                ? " tiles" + std::to_string(b->tile_rhs) + " cache" + std::to_string(b->cache_mb)
                                : std::string();
  hipEvent_t e0 = nullptr, e1 = nullptr;
  void* d_desc = nullptr;
  void* d_st = nullptr;
  const size_t desc_bytes = (size_t)nt * std::max(sizeof(tbs::RowArgs), sizeof(tbs::ColArgs));
  int rc = TBS_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess ||
      hipMalloc(&d_desc, desc_bytes) != hipSuccess || hipMalloc(&d_st, (size_t)nt * sizeof(int)) != hipSuccess) {
    (void)hipGetLastError();
    rc = bfail(b, TBS_ERR_OOM, "batch tuning buffers");
  }
  // time one grouped launch (2 warm-up, 3 timed)
  auto timeit = [&](auto&& launch) -> double {
    for (int w = 0; w < 2; ++w) launch();
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < 3; ++r) launch();
    (void)hipEventRecord(e1, s);
    if (hipEventSynchronize(e1) != hipSuccess) return 1e30;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    return ms / 3.0;
  };
  std::map<int, std::vector<int>> by_row;
  std::map<std::pair<int, int>, std::vector<int>> by_col;
  for (int i = 0; i < np; ++i) {
    by_row[(int)b->plans[i]->M[0]].push_back(i);
    by_col[{(int)b->plans[i]->M[1], b->plans[i]->cb}].push_back(i);
  }
  auto members_key = [&](const std::vector<int>& mem) {
    std::vector<std::string> parts;
    for (int i : mem)
      parts.push_back(std::to_string(b->plans[i]->N[0]) + "x" + std::to_string(b->plans[i]->N[1]) + "x" +
                      std::to_string(b->plans[i]->batch));
    std::sort(parts.begin(), parts.end());
    std::string k;
    for (const auto& q : parts) k += (k.empty() ? "" : ",") + q;
    return k;
  };
  // the tiles of each set and chain whose plan is one of mem: the launches
  // the solves make for one pass kind of one length
  auto set_tiles = [&](const std::vector<int>& mem) {
    std::vector<std::vector<int>> out((size_t)b->nsets * kMaxChains);
    for (int t = 0; t < nt; ++t)
      if (std::find(mem.begin(), mem.end(), b->tiles[t].plan) != mem.end())
        out[(size_t)b->tiles[t].set * kMaxChains + b->tiles[t].chain].push_back(t);
    return out;
  };
  // one candidate: every set's grouped launch of these tiles, timed and summed
  auto time_sets = [&](const std::vector<std::vector<int>>& sets, bool row, int M, int cb, int shape) -> double {
    double total_ms = 0.0;
    for (const auto& ts : sets) {
      if (ts.empty() || rc) continue;
      std::vector<int> st;
      int total = 0;
      std::vector<tbs::RowArgs> dr;
      std::vector<tbs::ColArgs> dc;
      for (int t : ts) {
        const int i = b->tiles[t].plan;
        st.push_back(total);
        if (row) {
          dr.push_back(tile_row_args(b, t, 2, 3, sources[i], potentials[i], p_outs[i]));
          total += row_blocks(b->plans[i]) * b->tiles[t].nrhs;
        } else {
          dc.push_back(tile_col_args(b, t));
          total += dc.back().nrhs * dc.back().n1 * dc.back().n0;
        }
      }
      const size_t db = row ? dr.size() * sizeof(tbs::RowArgs) : dc.size() * sizeof(tbs::ColArgs);
      if (hipMemcpy(d_desc, row ? (const void*)dr.data() : (const void*)dc.data(), db, hipMemcpyHostToDevice) !=
              hipSuccess ||
          hipMemcpy(d_st, st.data(), st.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipGetLastError();
        rc = bfail(b, TBS_ERR_HIP, "batch tuning tables");
        break;
      }
      int le = 0;
      total_ms += timeit([&] {
        const int e = row ? tbs::launch_row_group(b->fp64, M, cb, shape, (const tbs::RowArgs*)d_desc,
                                                  (const int*)d_st, (int)ts.size(), total, s)
                          : tbs::launch_col_group(b->fp64, M, shape, (const tbs::ColArgs*)d_desc,
                                                  (const int*)d_st, (int)ts.size(), total, s);
        if (e) le = e;
      });
      if (le) rc = bfail(b, TBS_ERR_HIP, std::string("batch tuning launch: ") + hipGetErrorString((hipError_t)le));
    }
    return total_ms;
  };
  // rows: one choice of rows per block for all plans of one x length
  for (auto it = by_row.begin(); !rc && it != by_row.end(); ++it) {
    const int M = it->first;
    const std::vector<int>& mem = it->second;
    int cand[8];
    const int n = tbs::row_nr_candidates(M, b->fp64, cand);
    const std::string key = "batchrow " + tag + " M" + std::to_string(M) + " " + members_key(mem) + sched;
    std::vector<int> v;
    int pick = cand[0];
    if (tune_lookup(key, &v) && v.size() == 1 && in_list(v[0], cand, n)) {
      pick = v[0];
    } else if (n > 1) {
      const auto sets = set_tiles(mem);
      double best = 1e30;
      for (int ci = 0; ci < n && !rc; ++ci) {
        for (int i : mem) b->plans[i]->row_nr = cand[ci];
        const double t = time_sets(sets, true, M, b->plans[mem[0]]->cb, cand[ci]);
        if (!rc && t < best) {
          best = t;
          pick = cand[ci];
        }
      }
      if (!rc) tune_store(key, {pick});
    }
    for (int i : mem) b->plans[i]->row_nr = pick;
  }
  // columns: one choice of columns per block for all plans of one y length
  for (auto it = by_col.begin(); !rc && it != by_col.end(); ++it) {
    const int M = it->first.first;
    const int cb = it->first.second;
    const std::vector<int>& mem = it->second;
    int cand[8];
    const int n = tbs::conv_nc_candidates(M, b->fp64, cb, cand);
    const std::string key = "batchcol " + tag + " M" + std::to_string(M) + " cb" + std::to_string(cb) + " " +
                            members_key(mem) + sched;
    std::vector<int> v;
    int pick = cand[0];
    if (tune_lookup(key, &v) && v.size() == 1 && in_list(v[0], cand, n)) {
      pick = v[0];
    } else if (n > 1) {
      const auto sets = set_tiles(mem);
      double best = 1e30;
      for (int ci = 0; ci < n && !rc; ++ci) {
        for (int i : mem) b->plans[i]->conv_nc = cand[ci];
        const double t = time_sets(sets, false, M, cb, cand[ci]);
        if (!rc && t < best) {
          best = t;
          pick = cand[ci];
        }
      }
      if (!rc) tune_store(key, {pick});
    }
    for (int i : mem) b->plans[i]->conv_nc = pick;
  }
  if (hipStreamSynchronize(s) != hipSuccess && !rc) rc = bfail(b, TBS_ERR_HIP, "batch tuning");
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (d_desc) (void)hipFree(d_desc);
  if (d_st) (void)hipFree(d_st);
  // launch chains of the cache-sized schedule (unless TBS_BATCH_CHAINS fixes
  // them): a short series (4 terms) per chain count, the second of two solves
  // (a graph replay) timed; one choice for the whole batch
  if (!rc && b->tile_rhs > 0 && !std::getenv("TBS_BATCH_CHAINS")) {
    std::vector<int> all(np);
    for (int i = 0; i < np; ++i) all[i] = i;
    const std::string key = "batchchains " + tag + " " + members_key(all) + sched;
    std::vector<int> v;
    int pick = b->chains;
    if (tune_lookup(key, &v) && v.size() == 1 && v[0] >= 1 && v[0] <= kMaxChains) {
      pick = v[0];
    } else {
      const hipStream_t cs = b->plans[0]->stream;
      hipEvent_t t0 = nullptr, t1 = nullptr;
      if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess) {
        (void)hipGetLastError();
        rc = bfail(b, TBS_ERR_HIP, "batch tuning events");
      }
      double best = 1e30;
      for (int K = 1; K <= kMaxChains && !rc; ++K) {
        b->chains = K;
        const int g = batch_group(b);
        if (g) {
          rc = bfail(b, g, "batch tables");
          break;
        }
        batch_drop_graph(b);
        float ms = 0.f;
        int e = tbs_batch_solve(b, sources, potentials, 4, p_outs, nullptr);
        if (e >= 0) {
          if (hipEventRecord(t0, cs) != hipSuccess) e = TBS_ERR_HIP;
          if (e >= 0) e = tbs_batch_solve(b, sources, potentials, 4, p_outs, nullptr);
          if (e >= 0 && (hipEventRecord(t1, cs) != hipSuccess || hipEventSynchronize(t1) != hipSuccess ||
                         hipEventElapsedTime(&ms, t0, t1) != hipSuccess))
            e = TBS_ERR_HIP;
        }
        if (e < 0) {
          rc = bfail(b, e, "batch chain tuning solve");
          break;
        }
        if (ms < best) {
          best = ms;
          pick = K;
        }
      }
      if (t0) (void)hipEventDestroy(t0);
      if (t1) (void)hipEventDestroy(t1);
      if (!rc) tune_store(key, {pick});
    }
    b->chains = pick;
  }
  // regroup with the chosen shapes (also after a failure: shapes may have moved)
  const int grc = batch_group(b);
  if (!rc && grc) rc = bfail(b, grc, "batch tables");
  if (!batch_sync(b) && !rc) rc = bfail(b, TBS_ERR_HIP, "batch tuning");
  batch_drop_graph(b);
  return rc;
}

int tbs_batch_profile_enable(tbs_batch* b, int enable) {
  if (!b) return TBS_ERR_INVALID;
  if (b->stream && hipStreamSynchronize(b->stream) != hipSuccess)
    return bfail(b, TBS_ERR_HIP, "batch: previous solve failed");
  b->prof = enable != 0;
  b->ev_used = 0;
  b->marks.clear();
  b->prof_ms.assign(3 * b->rgroups.size() + b->cgroups.size(), 0.0);
  b->prof_n.assign(b->prof_ms.size(), 0);
  return TBS_OK;
}

int tbs_batch_profile_read(tbs_batch* b, int cap, int* nentries, int* kind, int* length, int* shape,
                           int64_t* launches, double* ms, int* first, int* members, int* member_rhs) {
  if (!b || !nentries) return TBS_ERR_INVALID;
  const int nrg = (int)b->rgroups.size();
  const int ne = 3 * nrg + (int)b->cgroups.size();
  *nentries = ne;
  if (cap < ne) return bfail(b, TBS_ERR_INVALID, "profile arrays too short");
  if (hipStreamSynchronize(b->stream) != hipSuccess) return bfail(b, TBS_ERR_HIP, "batch: solve failed");
  if (b->prof_ms.size() != (size_t)ne) {
    b->prof_ms.assign(ne, 0.0);
    b->prof_n.assign(ne, 0);
  }
  for (const auto& m : b->marks) {
    float t = 0.0f;
    if (hipEventElapsedTime(&t, b->ev_pool[m.second], b->ev_pool[m.second + 1]) != hipSuccess)
      return bfail(b, TBS_ERR_HIP, "profile event time");
    b->prof_ms[m.first] += t;
    b->prof_n[m.first] += 1;
  }
  b->marks.clear();
  b->ev_used = 0;
  int off = 0;
  for (int e = 0; e < ne; ++e) {
    const bool row = e < 3 * nrg;
    const tbs_batch::Group& g = row ? b->rgroups[e / 3] : b->cgroups[e - 3 * nrg];
    if (kind) kind[e] = row ? e % 3 : 3;
    if (length) length[e] = g.M;
    if (shape) shape[e] = row ? (g.nr ? g.nr : tbs::row_rows_per_block(g.M, b->fp64)) : g.nc;
    if (launches) launches[e] = b->prof_n[e];
    if (ms) ms[e] = b->prof_ms[e];
    if (first) first[e] = off;
    for (int t : g.members) {
      if (members) members[off] = b->tiles[t].plan;
      if (member_rhs) member_rhs[off] = b->tiles[t].nrhs;
      ++off;
    }
    b->prof_ms[e] = 0.0;
    b->prof_n[e] = 0;
  }
  if (first) first[ne] = off;
  return TBS_OK;
}

void tbs_batch_destroy(tbs_batch* b) {
  if (!b) return;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  for (hipEvent_t ev : b->ev_pool) (void)hipEventDestroy(ev);
  batch_drop_graph(b);
  batch_free_tables(b);
  if (b->ev_in) (void)hipEventDestroy(b->ev_in);
  if (b->ev_out) (void)hipEventDestroy(b->ev_out);
  (void)batch_sync(b);
  if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
  for (int c = 1; c < kMaxChains; ++c) {
    if (b->ev_join[c]) (void)hipEventDestroy(b->ev_join[c]);
    if (b->cstream[c]) (void)hipStreamDestroy(b->cstream[c]);
  }
  if (b->stream) (void)hipStreamDestroy(b->stream);
  if (b->counted)
    for (tbs_plan* p : b->plans) p->batch_refs -= 1;
  delete b;
}

const char* tbs_batch_last_error(const tbs_batch* b) {
  if (!b) return g_create_err.c_str();
  return b->err.c_str();
}

const char* tbs_last_error(const tbs_plan* p) {
  if (!p) return g_create_err.c_str();
  return p->err.c_str();
}

}  // extern "C"

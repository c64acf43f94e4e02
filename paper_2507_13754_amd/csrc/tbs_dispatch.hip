// Length-family dispatch and the per-length configuration queries.
#include <algorithm>

#include "tbs_passes.hpp"

namespace tbs {

static int family(const PassReq& q, hipStream_t s) {
  switch (odd_part(q.M)) {
    case 1: return dispatch_pow2(q, s);
    case 3: return dispatch_three(q, s);
    case 5: return dispatch_five(q, s);
    default: return (int)hipErrorInvalidValue;
  }
}

int fft_supported_lengths(int* out, int cap) {
  int n = 0;
  int all[64];
#define TBS_ADD(m) all[n++] = m;
  TBS_LENGTHS_POW2(TBS_ADD) TBS_LENGTHS_THREE(TBS_ADD) TBS_LENGTHS_FIVE(TBS_ADD)
#undef TBS_ADD
  std::sort(all, all + n);
  for (int i = 0; i < n && i < cap; ++i) out[i] = all[i];
  return n;
}

bool fft_length_supported(int M) {
  int l[64];
  const int n = fft_supported_lengths(l, 64);
  return std::find(l, l + n, M) != l + n;
}

int fft_elems_per_thread(int M, bool fp64) { return elems_per_thread(M, fp64); }
int row_rows_per_block(int M, bool fp64) { return rows_per_block(M, fp64); }

// Contiguous spectral columns per block of the intermediate layout: 4, except
// FP64 with columns of 4096+ values.
int spectral_block(int My, bool fp64) { return (fp64 && My >= 4096) ? 2 : 4; }

int conv_cols_per_block(int M, bool fp64, int cb) {
  const int want = conv_default_cols(M, fp64);
  return want < cb ? want : cb;
}

int col_max_cols(int M, bool fp64) {
  const int esz = fp64 ? 16 : 8;
  (void)esz;
  return col_fits(M, 4, esz) ? 4 : (col_fits(M, 2, esz) ? 2 : 1);
}

int row_nr_candidates(int M, bool fp64, int* out) {
  const int esz = fp64 ? 16 : 8;
  int n = 0;
  out[n++] = rows_per_block(M, fp64);
  if (M >= 2048) {
    for (int nr : {2, 4})
      if (nr != out[0] && row_fits(M, nr, esz)) out[n++] = nr;
  }
  return n;
}

int conv_nc_candidates(int M, bool fp64, int cb, int* out) {
  const int esz = fp64 ? 16 : 8;
  int n = 0;
  out[n++] = conv_cols_per_block(M, fp64, cb);
  for (int nc : {1, 2, 4}) {
    if (nc == out[0] || nc > cb || cb % nc) continue;
    if (nc == 1 && M < 2048) continue;
    if (!col_fits(M, nc, esz)) continue;
    out[n++] = nc;
  }
  return n;
}

int launch_row_pass(bool fp64, int M, const RowArgs& a, int nblk_rows, int nr, hipStream_t s) {
  PassReq q;
  q.nr = nr;
  q.kind = PASS_ROW;
  q.fp64 = fp64;
  q.M = M;
  q.row = &a;
  q.nblk_rows = nblk_rows;
  return family(q, s);
}

int launch_col_pass(bool fp64, int M, int NC, const ColArgs& a, hipStream_t s) {
  PassReq q;
  q.kind = PASS_COL;
  q.fp64 = fp64;
  q.M = M;
  q.nc = NC;
  q.col = &a;
  return family(q, s);
}

int launch_row_fft_full(int M, void* data, const void* tw, int nrows, int inverse, hipStream_t s) {
  PassReq q;
  q.kind = PASS_ROW_FULL;
  q.fp64 = true;
  q.M = M;
  q.data = data;
  q.tw = tw;
  q.nrows = nrows;
  q.inverse = inverse;
  return family(q, s);
}

int launch_row_group(bool fp64, int M, int cb, int nr, const RowArgs* descs, const int* starts,
                     int ngroups, int total_blocks, hipStream_t s) {
  PassReq q;
  q.nr = nr;
  q.kind = PASS_ROW_GROUP;
  q.fp64 = fp64;
  q.M = M;
  q.cb = cb;
  q.row_descs = descs;
  q.starts = starts;
  q.ngroups = ngroups;
  q.total = total_blocks;
  return family(q, s);
}

int launch_col_group(bool fp64, int M, int nc, const ColArgs* descs, const int* starts, int ngroups,
                     int total_blocks, hipStream_t s) {
  PassReq q;
  q.kind = PASS_COL_GROUP;
  q.fp64 = fp64;
  q.M = M;
  q.nc = nc;
  q.col_descs = descs;
  q.starts = starts;
  q.ngroups = ngroups;
  q.total = total_blocks;
  return family(q, s);
}

}  // namespace tbs

// Host-side internals of libqc shared by the API translation units: the
// context, error reporting and the argument / device-side validation helpers.
#pragma once

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "qc_internal.h"

// Workgroups per compute unit that the automatic split aims at: the split
// passes are latency-bound, and the chain workload's terms (delay,
// bandpass, gain, direction-dependent) and the pointing and delay-offset
// solves ran 10-30% faster at about 32 than at 4 (measured; flat beyond).
constexpr int SPLIT_WG_PER_CU = 32;
// Wavefronts per compute unit that the split over one-channel intervals aims
// at (each holds 16 intervals and 24 KiB of LDS at 64 antennas, so about six
// are resident per CU: two rounds of them; 6 to 48 measured within 6%)
constexpr int BAND_WAVES_PER_CU = 12;

struct qc_ctx {
  int device = 0;
  std::string msg;
  hipStream_t last_stream = nullptr;
  int* d_err = nullptr;
  long long* d_rowpos = nullptr;
  size_t rowpos_cap = 0;
  long long* d_rowlo = nullptr;
  size_t rowlo_cap = 0;
  long long* d_rowhi = nullptr;
  size_t rowhi_cap = 0;
  int* d_tt = nullptr;        // [2][n_gt] time range per gain time
  size_t tt_cap = 0;
  int* d_chlo = nullptr;
  size_t chlo_cap = 0;
  int* d_chhi = nullptr;
  size_t chhi_cap = 0;
  int max_int_chan = 0;       // channels of the widest interval of the last prepared term
  std::vector<int> h_clo, h_chi;   // channel range of every interval of the last prepared term
  float* d_dh = nullptr;      // MLP backward scratch [batch][n_hid]
  size_t dh_cap = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  bool timed = false;
  int waves = 4;              // waves per workgroup of the per-interval solve
  int rows_per_step = 0;      // 0: the kernel default
  int split_parts = 0;        // 0: automatic, 1: never split, > 1: parts per interval
  int n_cu = 0;               // compute units of the device
  double* d_partials = nullptr;
  size_t partials_cap = 0;
  unsigned char* d_otab = nullptr;    // fixed chain factors of diagonal chains
  size_t otab_cap = 0;
  // MAD flagging scratch
  unsigned char* d_fl_stat = nullptr;  // per-sample statistic
  size_t fl_stat_cap = 0;
  unsigned char* d_fl_groups = nullptr;
  size_t fl_groups_cap = 0;
  unsigned* d_fl_hist = nullptr;
  size_t fl_hist_cap = 0;
  int* d_fl_count = nullptr;
  size_t fl_count_cap = 0;
  int* d_fl_rows = nullptr;
  size_t fl_rows_cap = 0;
  unsigned long long* d_fl_new = nullptr;
  size_t fl_new_cap = 0;
  double* d_rw = nullptr;              // robust reweighting: partial sums, s2
  size_t rw_cap = 0;
  unsigned char* d_pc = nullptr;       // prepared sky components, direction order
  size_t pc_cap = 0;
  int* d_pc_off = nullptr;             // [n_dir + 1] first component of each direction
  size_t pc_off_cap = 0;
  double* d_dv = nullptr;              // split schedule: divergence state per block
  size_t dv_cap = 0;
  int* d_passes = nullptr;
  size_t passes_cap = 0;
  uint8_t* d_done = nullptr;
  size_t done_cap = 0;
  int* d_active = nullptr;
  size_t active_cap = 0;
  int* d_pt_int = nullptr;             // pointing solves: iterations, done, divergence runs
  size_t pt_int_cap = 0;
  double* d_pt_dbl = nullptr;          // pointing solves: chi^2 first/last, previous steps
  size_t pt_dbl_cap = 0;
  double* d_lm = nullptr;              // split schedule, Levenberg-Marquardt: state per interval
  size_t lm_cap = 0;
  double2* d_acc = nullptr;            // split schedule, Levenberg-Marquardt: last accepted gains
  size_t acc_cap = 0;
  qc::BandStep* d_band = nullptr;        // split schedule over one-channel intervals: steps per row
  size_t band_cap = 0;
  unsigned char* d_ddtab = nullptr;    // that split: tables of the direction-dependent fixed terms
  size_t ddtab_cap = 0;
  int last_split_parts = 1;   // parts per interval of the last solve (1 = fused)
  unsigned char* static_scratch = nullptr;   // this device's allocation-free scratch array (qc_api.hip)
};

namespace qc {

inline qc_status fail(qc_ctx* ctx, qc_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (ctx) ctx->msg = buf;
  return st;
}

#define HIP_TRY(ctx, expr)                                                                   \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return fail(ctx, e_ == hipErrorOutOfMemory ? QC_E_NOMEM : QC_E_DEVICE, "%s: %s", #expr, \
                  hipGetErrorString(e_));                                                    \
  } while (0)

template <typename P>
hipError_t grow(P*& ptr, size_t& cap, size_t n) {
  if (n <= cap && ptr) return hipSuccess;
  if (ptr) {
    hipError_t e = hipFree(ptr);
    if (e != hipSuccess) return e;
    ptr = nullptr;
  }
  size_t want = std::max<size_t>(n, 64);
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&ptr), want * sizeof(P));
  if (e != hipSuccess) {
    cap = 0;
    ptr = nullptr;
    return e;
  }
  cap = want;
  return hipSuccess;
}


struct HostMaps {
  std::vector<int> t_map, f_map, d_map;
};

// Device scratch of the argument checks and interval ranges: the row position
// of every time [n_time + 1], the row range [n_gt] x 2 and time range [2][n_gt]
// of every gain time and the channel range [n_gf] x 2 of every gain frequency
// of the active term.
struct PrepScratch {
  long long* rowpos = nullptr;
  long long* rowlo = nullptr;
  long long* rowhi = nullptr;
  int* tt = nullptr;
  int* chlo = nullptr;
  int* chhi = nullptr;
};

// Checks the visibilities and the chain, validates the rows on the device and
// (active >= 0) computes the interval ranges of the active term, into `fixed`
// when given, else into the context's scratch (grown as needed); waits for
// the device checks.
// need_model false: vis->model may be NULL (a model predicted from a sky).
qc_status prepare(qc_ctx* ctx, const qc_vis* v, const qc_term* chain, int n_term, int active,
                  std::vector<HostMaps>& maps, hipStream_t s, const PrepScratch* fixed = nullptr,
                  bool need_model = true);
void fill_args(const qc_vis* v, const qc_term* chain, int n_term, int active, VisArgs& va, ChainArgs& ca);
qc_status read_err(qc_ctx* ctx, hipStream_t s);
// check_vis plus the device checks of row order and antenna/time ranges
// (waits for them); for calls that take no chain
qc_status validate_rows(qc_ctx* ctx, const qc_vis* v, hipStream_t s);
int resolve_damping(qc_damping d, const qc_term& t);
// the schedule of an active pointing term (after prepare())
qc_status solve_pointing(qc_ctx* ctx, const qc_vis* vis, qc_term* chain, int n_term, int active,
                         const qc_solve_opts* opts, qc_solve_stats* stats, hipStream_t s);
bool dmap_constant(const HostMaps& hm);
// Checks a point-component sky and prepares its table (direction order, the
// context's memory) for n_dir model directions; uvw [n_row][3] (device) is
// carried along.  Waits for `s`.
qc_status prepare_sky(qc_ctx* ctx, const qc_sky* sky, int n_dir, const double* uvw, hipStream_t s, SkyArgs& out);

}  // namespace qc

// Host side of the libqc C-ABI: context, argument checks, the device-side
// validation pre-pass (row order, antenna and time ranges, per-interval row
// ranges) and the public entry points declared in include/qc.h.

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "qc_host.h"
#include "qc_hostcheck.h"

using namespace qc;

namespace qc {

// ---------------------------------------------------------------------------
// validation kernels
// ---------------------------------------------------------------------------

__global__ void k_clear(int* err) {
  if (threadIdx.x == 0 && blockIdx.x == 0) err[0] = 0;
}

// For rows sorted by time, rowpos[t] = first row with row_time >= t
// (t = 0 .. n_time).  Each entry is written by exactly one row when the
// order is valid; bad input raises a flag and every write stays in bounds.
__global__ void k_rows(VisArgs v, long long* rowpos, int* err) {
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= v.n_row) return;
  const int nt = v.n_time;
  int t = v.row_time[r];
  const int p = v.ant1[r], q = v.ant2[r];
  int bad = 0;
  if ((unsigned)p >= (unsigned)v.n_ant || (unsigned)q >= (unsigned)v.n_ant) bad |= ERR_RANGE;
  if ((unsigned)t >= (unsigned)nt) bad |= ERR_RANGE;
  int tp = (r > 0) ? v.row_time[r - 1] : -1;
  if (r > 0 && tp > t) bad |= ERR_ORDER;
  if (bad) atomicOr(err, bad);
  t = min(max(t, -1), nt - 1);
  tp = min(max(tp, -1), nt - 1);
  for (int tt = tp + 1; tt <= t; ++tt) rowpos[tt] = r;
  if (r == v.n_row - 1)
    for (int tt = max(t, -1) + 1; tt <= nt; ++tt) rowpos[tt] = v.n_row;
}

__global__ void k_rowpos_empty(long long* rowpos, int nt) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t <= nt) rowpos[t] = 0;
}

__global__ void k_ranges(const long long* rowpos, const int* tt, int n_gt, long long* lo, long long* hi) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_gt) return;
  lo[g] = rowpos[tt[g]];
  hi[g] = rowpos[tt[n_gt + g]];
}

// ---------------------------------------------------------------------------
// host checks
// ---------------------------------------------------------------------------

qc_status check_vis(qc_ctx* ctx, const qc_vis* v, bool need_model) {
  const Check c = check_vis_fields(v, need_model);
  return c.st == QC_OK ? QC_OK : fail(ctx, c.st, "%s", c.msg.c_str());
}

qc_status check_term(qc_ctx* ctx, const qc_vis* v, const qc_term* t, int j, HostMaps& hm, hipStream_t s) {
  Check c = check_term_fields(t, j);
  if (c.st != QC_OK) return fail(ctx, c.st, "%s", c.msg.c_str());
  if (t->type == QC_TERM_POINTING) {
    std::vector<double> lm(2 * (size_t)v->n_dir);
    HIP_TRY(ctx, hipMemcpyAsync(lm.data(), t->dir_lm, sizeof(double) * lm.size(), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    c = check_dir_lm(lm.data(), v->n_dir, j);
    if (c.st != QC_OK) return fail(ctx, c.st, "%s", c.msg.c_str());
  }
  hm.t_map.resize(v->n_time);
  hm.f_map.resize(v->n_chan);
  hm.d_map.resize(v->n_dir);
  HIP_TRY(ctx, hipMemcpyAsync(hm.t_map.data(), t->t_map, sizeof(int) * v->n_time, hipMemcpyDeviceToHost, s));
  HIP_TRY(ctx, hipMemcpyAsync(hm.f_map.data(), t->f_map, sizeof(int) * v->n_chan, hipMemcpyDeviceToHost, s));
  HIP_TRY(ctx, hipMemcpyAsync(hm.d_map.data(), t->d_map, sizeof(int) * v->n_dir, hipMemcpyDeviceToHost, s));
  HIP_TRY(ctx, hipStreamSynchronize(s));
  c = check_term_maps(t, j, hm.t_map.data(), v->n_time, hm.f_map.data(), v->n_chan, hm.d_map.data(), v->n_dir);
  return c.st == QC_OK ? QC_OK : fail(ctx, c.st, "%s", c.msg.c_str());
}

bool dmap_constant(const HostMaps& hm) {
  for (size_t i = 1; i < hm.d_map.size(); ++i)
    if (hm.d_map[i] != hm.d_map[0]) return false;
  return true;
}

void fill_args(const qc_vis* v, const qc_term* chain, int n_term, int active, VisArgs& va, ChainArgs& ca) {
  va.data = v->data;
  va.model = v->model;
  va.weight = v->weight;
  va.flag = v->flag;
  va.ant1 = v->ant1;
  va.ant2 = v->ant2;
  va.row_time = v->row_time;
  va.freq = v->chan_freq;
  va.n_row = v->n_row;
  va.n_chan = v->n_chan;
  va.n_dir = v->n_dir;
  va.n_ant = v->n_ant;
  va.n_time = v->n_time;
  va.n_wcorr = v->n_wcorr;
  memset(&ca, 0, sizeof ca);
  ca.n_term = n_term;
  ca.active = active;
  for (int j = 0; j < n_term; ++j) {
    const qc_term& t = chain[j];
    TermArgs& ta = ca.t[j];
    ta.kind = (int)t.type;
    ta.n_gt = t.n_gt;
    ta.n_gf = t.n_gf;
    ta.n_gdir = t.n_gdir;
    ta.t_map = t.t_map;
    ta.f_map = t.f_map;
    ta.d_map = t.d_map;
    ta.gains = reinterpret_cast<const double2*>(t.gains);
    ta.params = t.params;
    if (t.type == QC_TERM_POINTING) {
      // one parameter pair per antenna, a gain per model direction: every chain
      // path treats the term as direction dependent
      ta.n_gdir = v->n_dir;
      ta.dir_lm = t.dir_lm;
      ta.beta = 4.0 * std::log(2.0) / ((t.beam_fwhm * t.beam_freq) * (t.beam_fwhm * t.beam_freq));
    }
  }
}

qc_status read_err(qc_ctx* ctx, hipStream_t s) {
  int h = 0;
  HIP_TRY(ctx, hipMemcpyAsync(&h, ctx->d_err, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(ctx, hipStreamSynchronize(s));
  if (h & ERR_ORDER) return fail(ctx, QC_E_ARG, "row_time is not non-decreasing");
  if (h & ERR_RANGE) return fail(ctx, QC_E_RANGE, "antenna or time index out of range");
  if (h & ERR_NONFINITE) return fail(ctx, QC_E_NONFINITE, "non-finite value in an unflagged sample");
  return QC_OK;
}

// Validates the rows on the device and (when active >= 0) computes the row
// and channel ranges of every solution interval of the active term.
qc_status validate_rows(qc_ctx* ctx, const qc_vis* v, hipStream_t s) {
  qc_status st = check_vis(ctx, v, true);
  if (st != QC_OK) return st;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  VisArgs va;
  ChainArgs ca;
  fill_args(v, nullptr, 0, -1, va, ca);
  HIP_TRY(ctx, grow(ctx->d_rowpos, ctx->rowpos_cap, (size_t)v->n_time + 1));
  hipLaunchKernelGGL(k_clear, dim3(1), dim3(64), 0, s, ctx->d_err);
  if (v->n_row > 0) {
    const long long nb = (v->n_row + 255) / 256;
    hipLaunchKernelGGL(k_rows, dim3((unsigned)nb), dim3(256), 0, s, va, ctx->d_rowpos, ctx->d_err);
  }
  HIP_TRY(ctx, hipGetLastError());
  return read_err(ctx, s);
}

qc_status prepare(qc_ctx* ctx, const qc_vis* v, const qc_term* chain, int n_term, int active,
                  std::vector<HostMaps>& maps, hipStream_t s, const PrepScratch* fixed, bool need_model) {
  qc_status st = check_vis(ctx, v, need_model);
  if (st != QC_OK) return st;
  if (!chain || n_term <= 0) return fail(ctx, QC_E_ARG, "empty chain");
  if (n_term > QC_MAX_TERMS) return fail(ctx, QC_E_UNSUPPORTED, "n_term=%d exceeds %d", n_term, QC_MAX_TERMS);
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  maps.assign(n_term, HostMaps());
  for (int j = 0; j < n_term; ++j) {
    st = check_term(ctx, v, &chain[j], j, maps[j], s);
    if (st != QC_OK) return st;
  }
  VisArgs va;
  ChainArgs ca;
  fill_args(v, chain, n_term, active, va, ca);
  // device scratch: the context's (grown as needed) or the caller's fixed block
  PrepScratch sc;
  if (fixed) {
    sc = *fixed;
  } else {
    HIP_TRY(ctx, grow(ctx->d_rowpos, ctx->rowpos_cap, (size_t)v->n_time + 1));
    sc.rowpos = ctx->d_rowpos;
  }
  hipLaunchKernelGGL(k_clear, dim3(1), dim3(64), 0, s, ctx->d_err);
  if (v->n_row > 0) {
    const long long nb = (v->n_row + 255) / 256;
    hipLaunchKernelGGL(k_rows, dim3((unsigned)nb), dim3(256), 0, s, va, sc.rowpos, ctx->d_err);
  } else {
    hipLaunchKernelGGL(k_rowpos_empty, dim3((v->n_time + 256) / 256), dim3(256), 0, s, sc.rowpos, v->n_time);
  }
  HIP_TRY(ctx, hipGetLastError());
  if (active >= 0) {
    const qc_term& ta = chain[active];
    const HostMaps& hm = maps[active];
    std::vector<int> tt, clo, chi;
    ctx->max_int_chan = interval_extents(hm.t_map, hm.f_map, ta.n_gt, ta.n_gf, tt, clo, chi);
    if (!fixed) {
      HIP_TRY(ctx, grow(ctx->d_rowlo, ctx->rowlo_cap, (size_t)ta.n_gt));
      HIP_TRY(ctx, grow(ctx->d_rowhi, ctx->rowhi_cap, (size_t)ta.n_gt));
      HIP_TRY(ctx, grow(ctx->d_tt, ctx->tt_cap, 2 * (size_t)ta.n_gt));
      HIP_TRY(ctx, grow(ctx->d_chlo, ctx->chlo_cap, (size_t)ta.n_gf));
      HIP_TRY(ctx, grow(ctx->d_chhi, ctx->chhi_cap, (size_t)ta.n_gf));
      sc.rowlo = ctx->d_rowlo;
      sc.rowhi = ctx->d_rowhi;
      sc.tt = ctx->d_tt;
      sc.chlo = ctx->d_chlo;
      sc.chhi = ctx->d_chhi;
    }
    ctx->h_clo = clo;
    ctx->h_chi = chi;
    HIP_TRY(ctx, hipMemcpyAsync(sc.tt, tt.data(), sizeof(int) * tt.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(ctx, hipMemcpyAsync(sc.chlo, clo.data(), sizeof(int) * clo.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(ctx, hipMemcpyAsync(sc.chhi, chi.data(), sizeof(int) * chi.size(), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_ranges, dim3((ta.n_gt + 255) / 256), dim3(256), 0, s, sc.rowpos, sc.tt, ta.n_gt,
                       sc.rowlo, sc.rowhi);
    HIP_TRY(ctx, hipGetLastError());
  }
  return read_err(ctx, s);
}

int resolve_damping(qc_damping d, const qc_term& t) {
  if (d == QC_DAMP_AUTO) {
    // full steps for delay and phase-only terms: a common phase or delay
    // leaves the model unchanged, so there is no scale mode to overshoot
    if (t.type == QC_TERM_DELAY || t.type == QC_TERM_PHASE || t.type == QC_TERM_DELAY_OFFSET) return 0;
    // pointing: the beams enter the model as the product b_p b_q (as amplitudes do)
    if (t.type == QC_TERM_POINTING) return 2;
    return t.direction_dependent ? 1 : 2;
  }
  return (int)d;
}

}  // namespace qc

// ---------------------------------------------------------------------------
// allocation-free scratch (qc_solve_interval_static)
// ---------------------------------------------------------------------------

// A fixed device array for the scratch of qc_solve_interval_static: each
// device that loads the library holds its own copy until the process ends.
// Host code never passes the array's name to a kernel or a copy (on the host
// it is a stand-in, not a device address): it uses the address that
// hipGetSymbolAddress returns for the current device, kept per device.
static __device__ __align__(256) unsigned char scratch[QC_STATIC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[MAX_DEVICES] = {};

// The address of this device's scratch array, looked up once per device
// with the device current.
qc_status static_scratch_ptr(int device, unsigned char** out) {
  if (device < 0 || device >= MAX_DEVICES) return QC_E_DEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return QC_E_DEVICE;
    g_scratch_ptr[device] = reinterpret_cast<unsigned char*>(p);
  }
  *out = g_scratch_ptr[device];
  return QC_OK;
}

// Carves the prepare scratch of a solve out of the static array; returns the
// bytes it needs (those beyond QC_STATIC_SCRATCH_BYTES are not carved).
size_t carve_static(unsigned char* base, const qc_vis* v, const qc_term& ta, PrepScratch& sc) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    unsigned char* p = base + off;
    off += (bytes + 255) & ~size_t(255);
    return p;
  };
  const size_t n_time = v ? (size_t)std::max(v->n_time, 0) : 0;
  const size_t n_gt = (size_t)std::max(ta.n_gt, 0), n_gf = (size_t)std::max(ta.n_gf, 0);
  sc.rowpos = reinterpret_cast<long long*>(take(sizeof(long long) * (n_time + 1)));
  sc.rowlo = reinterpret_cast<long long*>(take(sizeof(long long) * n_gt));
  sc.rowhi = reinterpret_cast<long long*>(take(sizeof(long long) * n_gt));
  sc.tt = reinterpret_cast<int*>(take(sizeof(int) * 2 * n_gt));
  sc.chlo = reinterpret_cast<int*>(take(sizeof(int) * n_gf));
  sc.chhi = reinterpret_cast<int*>(take(sizeof(int) * n_gf));
  return off;
}

}  // namespace

// ---------------------------------------------------------------------------
// public API
// ---------------------------------------------------------------------------

extern "C" {

qc_status qc_ctx_create(int32_t device, qc_ctx** out) {
  if (!out) return QC_E_ARG;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return QC_E_DEVICE;
  if (hipSetDevice(device) != hipSuccess) return QC_E_DEVICE;
  qc_ctx* c = new qc_ctx();
  c->device = device;
  if (hipMalloc(reinterpret_cast<void**>(&c->d_err), sizeof(int) * 4) != hipSuccess) {
    delete c;
    return QC_E_NOMEM;
  }
  hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, device);
  if (c->n_cu <= 0) c->n_cu = 256;
  if (static_scratch_ptr(device, &c->static_scratch) != QC_OK) {
    hipFree(c->d_err);
    delete c;
    return QC_E_DEVICE;
  }
  if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess) {
    hipFree(c->d_err);
    delete c;
    return QC_E_DEVICE;
  }
  *out = c;
  return QC_OK;
}

qc_status qc_ctx_destroy(qc_ctx* ctx) {
  if (!ctx) return QC_E_ARG;
  hipSetDevice(ctx->device);
  hipDeviceSynchronize();
  hipFree(ctx->d_err);
  hipFree(ctx->d_rowpos);
  hipFree(ctx->d_rowlo);
  hipFree(ctx->d_rowhi);
  hipFree(ctx->d_tt);
  hipFree(ctx->d_chlo);
  hipFree(ctx->d_chhi);
  hipFree(ctx->d_dh);
  hipFree(ctx->d_partials);
  hipFree(ctx->d_otab);
  hipFree(ctx->d_fl_stat);
  hipFree(ctx->d_fl_groups);
  hipFree(ctx->d_fl_hist);
  hipFree(ctx->d_fl_count);
  hipFree(ctx->d_fl_rows);
  hipFree(ctx->d_fl_new);
  hipFree(ctx->d_rw);
  hipFree(ctx->d_pc);
  hipFree(ctx->d_pc_off);
  hipFree(ctx->d_dv);
  hipFree(ctx->d_passes);
  hipFree(ctx->d_done);
  hipFree(ctx->d_active);
  hipFree(ctx->d_pt_int);
  hipFree(ctx->d_pt_dbl);
  hipFree(ctx->d_lm);
  hipFree(ctx->d_acc);
  hipFree(ctx->d_band);
  hipFree(ctx->d_ddtab);
  hipEventDestroy(ctx->ev0);
  hipEventDestroy(ctx->ev1);
  delete ctx;
  return QC_OK;
}

qc_status qc_ctx_sync(qc_ctx* ctx) {
  if (!ctx) return QC_E_ARG;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->last_stream));
  qc_status st = read_err(ctx, ctx->last_stream);
  hipLaunchKernelGGL(k_clear, dim3(1), dim3(64), 0, ctx->last_stream, ctx->d_err);
  HIP_TRY(ctx, hipStreamSynchronize(ctx->last_stream));
  return st;
}

const char* qc_last_error(const qc_ctx* ctx) { return ctx ? ctx->msg.c_str() : "null context"; }

double qc_last_kernel_ms(qc_ctx* ctx) {
  if (!ctx || !ctx->timed) return -1.0;
  if (hipEventSynchronize(ctx->ev1) != hipSuccess) return -1.0;
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1) != hipSuccess) return -1.0;
  return (double)ms;
}

}  // extern "C"

// qc_solve_interval; fixed != NULL: the allocation-free form (prepare scratch
// in `fixed`, always the fused schedule, no fixed-factor table, no pointing);
// sky != NULL: the model predicted from point components in the passes
static qc_status solve_interval_impl(qc_ctx* ctx, const qc_vis* vis, qc_term* chain, int32_t n_term,
                                     int32_t active, const qc_solve_opts* opts, qc_solve_stats* stats,
                                     const PrepScratch* fixed, const qc_sky* sky = nullptr,
                                     const double* uvw = nullptr) {
  if (!ctx) return QC_E_ARG;
  if (!opts) return fail(ctx, QC_E_ARG, "opts is NULL");
  if (!chain || n_term <= 0 || active < 0 || active >= n_term)
    return fail(ctx, QC_E_ARG, "active=%d outside the chain of %d terms", active, n_term);
  const int prec_v = enum_value(opts->prec), damp_v = enum_value(opts->damping);
  if (prec_v != QC_PREC_FP64 && prec_v != QC_PREC_MIXED) return fail(ctx, QC_E_ARG, "bad precision %d", prec_v);
  if (damp_v < QC_DAMP_FULL || damp_v > QC_DAMP_LM) return fail(ctx, QC_E_ARG, "bad damping %d", damp_v);
  if (opts->max_iter < 0) return fail(ctx, QC_E_ARG, "max_iter < 0");
  if (vis && prec_v == QC_PREC_MIXED && enum_value(vis->dtype) != QC_C64)
    return fail(ctx, QC_E_ARG, "MIXED precision needs complex64 data");
  hipStream_t s = reinterpret_cast<hipStream_t>(opts->stream);
  ctx->last_stream = s;
  if (fixed && enum_value(chain[active].type) == QC_TERM_POINTING)
    return fail(ctx, QC_E_UNSUPPORTED, "the allocation-free solve takes no active POINTING term");
  if (sky) {
    if (!uvw && vis && vis->n_row > 0) return fail(ctx, QC_E_ARG, "uvw is NULL");
    bool diag = true;
    for (int j = 0; j < n_term; ++j)
      if (enum_value(chain[j].type) == QC_TERM_COMPLEX2X2) diag = false;
    const bool single = vis && n_term == 1 && vis->n_dir == 1 && chain[active].n_gdir == 1;
    if (!single && !diag)
      return fail(ctx, QC_E_UNSUPPORTED, "the predicted model takes a single term or a chain of diagonal terms");
    if (enum_value(chain[active].type) == QC_TERM_POINTING)
      return fail(ctx, QC_E_UNSUPPORTED, "the predicted model takes no active POINTING term");
    if (damp_v == QC_DAMP_LM)
      return fail(ctx, QC_E_UNSUPPORTED, "the predicted model takes no Levenberg-Marquardt damping");
  }
  std::vector<HostMaps> maps;
  qc_status st = prepare(ctx, vis, chain, n_term, active, maps, s, fixed, sky == nullptr);
  if (st != QC_OK) return st;
  SkyArgs sk;
  memset(&sk, 0, sizeof sk);
  if (sky) {
    st = prepare_sky(ctx, sky, vis->n_dir, uvw, s, sk);
    if (st != QC_OK) return st;
  }
  if (chain[active].type == QC_TERM_POINTING)
    return solve_pointing(ctx, vis, chain, n_term, active, opts, stats, s);
  SolveLaunch L;
  memset(&L, 0, sizeof L);
  fill_args(vis, chain, n_term, active, L.vis, L.chain);
  L.vis_is_c128 = vis->dtype == QC_C128;
  L.prec_mixed = opts->prec == QC_PREC_MIXED;
  L.diag_chain = 1;
  for (int j = 0; j < n_term; ++j)
    if (chain[j].type == QC_TERM_COMPLEX2X2) L.diag_chain = 0;
  // A chain of diagonal terms commutes, so its diagonal-chain evaluation takes
  // any left factor (direction-dependent ones and pointing beams included).
  // Otherwise a left factor that is not diagonal, or differs by direction,
  // needs the full per-antenna blocks (eq. jonesfactor, eq. g_derivative_dd).
  L.left_general = 0;
  if (!L.diag_chain)
    for (int j = 0; j < active; ++j)
      if (chain[j].type == QC_TERM_COMPLEX2X2 || chain[j].type == QC_TERM_POINTING || !dmap_constant(maps[j]))
        L.left_general = 1;
  qc_term& ta = chain[active];
  L.gains = reinterpret_cast<double2*>(ta.gains);
  L.params = ta.params;
  L.gflags = ta.gain_flags;
  L.row_lo = fixed ? fixed->rowlo : ctx->d_rowlo;
  L.row_hi = fixed ? fixed->rowhi : ctx->d_rowhi;
  L.chan_lo = fixed ? fixed->chlo : ctx->d_chlo;
  L.chan_hi = fixed ? fixed->chhi : ctx->d_chhi;
  if (stats) {
    L.iters = stats->iters;
    L.converged = stats->converged;
    L.chisq_first = stats->chisq_first;
    L.chisq_last = stats->chisq_last;
    L.restarted = stats->restarted;
  }
  L.chisq_ref = opts->chisq_ref;
  L.sky = sk;
  L.tol = opts->tol;
  L.max_iter = opts->max_iter;
  L.damping = resolve_damping(opts->damping, ta);
  L.err = ctx->d_err;
  L.waves = ctx->waves;
  L.max_int_chan = ctx->max_int_chan;
  L.dir_ident = ta.n_gdir > 1 && ta.n_gdir == vis->n_dir && ta.n_gdir <= 4;
  for (int d = 0; L.dir_ident && d < vis->n_dir; ++d)
    if (maps[active].d_map[d] != d) L.dir_ident = 0;
  L.rows_per_step = ctx->rows_per_step == 8 ? 0 : ctx->rows_per_step;   // 8: the one-channel split only
  // schedule: fused (one workgroup per interval) unless the term has too few
  // intervals to give every CU several workgroups and they are large enough
  // (>= 2^18 samples on average) to amortise a host wait per iteration; those
  // are cut into parts streamed by separate workgroups (about SPLIT_WG_PER_CU per CU)
  const int n_int = ta.n_gt * ta.n_gf;
  const double avg_samples = n_int > 0 ? (double)vis->n_row * vis->n_chan / n_int : 0.0;
  int parts = 1;
  const bool lm = opts->damping == QC_DAMP_LM;
  if (lm && ta.type == QC_TERM_DELAY_OFFSET)
    return fail(ctx, QC_E_UNSUPPORTED, "Levenberg-Marquardt takes no delay-and-offset term");
  if (fixed) {
    parts = 1;                                 // the split schedule's state is context memory
  } else if (ctx->split_parts > 1) {
    parts = ctx->split_parts;
  } else if (ctx->split_parts == 0 && !opts->chisq_ref && n_int > 0 && n_int < 4 * ctx->n_cu &&
             avg_samples >= (double)(1 << 18)) {
    const double rows_per_int = (double)vis->n_row / std::max(ta.n_gt, 1);
    parts = (int)std::ceil((double)SPLIT_WG_PER_CU * ctx->n_cu / n_int);
    parts = std::max(2, std::min(parts, (int)std::max(1.0, rows_per_int / 64.0)));
  }
  if (parts > 1 && opts->chisq_ref)
    return fail(ctx, QC_E_UNSUPPORTED, "the split schedule does not take chisq_ref");
  // intervals of one channel each, in channel order, on a diagonal chain with
  // one gain direction: the split pass over 16 channels per wavefront
  bool band = parts > 1 && !sky && L.diag_chain && !L.left_general && ta.type == QC_TERM_DIAGONAL &&
              ta.n_gdir == 1 && ctx->max_int_chan == 1 && ta.n_gf == vis->n_chan && vis->n_row < (1LL << 31) &&
              band_lds_bytes_for(vis->n_ant, L.prec_mixed != 0, 8) <= 64 * 1024;
  for (int g = 0; band && g < ta.n_gf; ++g)
    if (ctx->h_clo[g] != g) band = false;
  // diagonal chains: the direction-dependent fixed terms, when all are
  // diagonal gains and at most BAND_MAX_DD, tabulated once per solve for every
  // pass (the band pass takes no other kind).  A pointing term differs by
  // direction through its beam although it has one gain direction.
  L.n_dd = 0;
  L.dd_tabled = !fixed && L.diag_chain && !L.left_general;
  for (int j = 0; L.dd_tabled && j < n_term; ++j) {
    const bool dd = chain[j].n_gdir > 1 || enum_value(chain[j].type) == QC_TERM_POINTING;
    if (j == active || !dd) continue;
    if (chain[j].type != QC_TERM_DIAGONAL || L.n_dd == BAND_MAX_DD) L.dd_tabled = 0;
    else L.dd_term[L.n_dd++] = j;
  }
  if (!L.dd_tabled) L.n_dd = 0;
  if (!L.dd_tabled) band = false;
  // 4 rows x 16 channels per step (measured faster than 8 x 8 on the 64-antenna
  // bandpass: 11.1 against 12.9 ms per pass), unless asked otherwise or its LDS
  // slots do not fit
  L.band_rows = (ctx->rows_per_step == 8 || band_lds_bytes_for(vis->n_ant, L.prec_mixed != 0, 4) > 64 * 1024) ? 8 : 4;
  if (band && ctx->split_parts == 0) {
    const long long units = (long long)((vis->n_chan + 64 / L.band_rows - 1) / (64 / L.band_rows)) * ta.n_gt;
    const double rows_per_int = (double)vis->n_row / std::max(ta.n_gt, 1);
    parts = (int)std::ceil((double)BAND_WAVES_PER_CU * ctx->n_cu / (double)units);
    parts = std::max(2, std::min(parts, (int)std::max(1.0, rows_per_int / 64.0)));
  }
  ctx->last_split_parts = parts;
  // diagonal chains: the direction-independent terms other than the active
  // one are fixed during the solve; tabulate their product once
  const bool single_chain = (n_term == 1 && vis->n_dir == 1 && ta.n_gdir == 1);
  bool other_di = false;
  for (int j = 0; j < n_term; ++j)
    if (j != active && chain[j].n_gdir == 1) other_di = true;
  const bool want_tab = !fixed && L.diag_chain && !single_chain && other_di;
  L.otab = nullptr;
  if (want_tab) HIP_TRY(ctx, grow(ctx->d_otab, ctx->otab_cap, chain_table_bytes(L)));
  SplitLaunch P;
  if (parts > 1) {
    // values per block (qc_interval.h: KindInfo NV, or NV_FB for full blocks)
    const int nv = L.left_general ? (ta.type == QC_TERM_DIAGONAL ? 8
                                     : ta.type == QC_TERM_COMPLEX2X2 ? 24 : (ta.type == QC_TERM_DELAY_OFFSET ? 14 : 5))
                                  : (ta.type == QC_TERM_DIAGONAL ? 6
                                     : ta.type == QC_TERM_COMPLEX2X2 ? 16 : (ta.type == QC_TERM_DELAY_OFFSET ? 10 : 4));
    const int ng = ta.n_gdir == 1 ? 1 : 4;
    const size_t stride = (size_t)vis->n_ant * ng * nv + 1;
    HIP_TRY(ctx, grow(ctx->d_partials, ctx->partials_cap, stride * (size_t)n_int * parts));
    HIP_TRY(ctx, grow(ctx->d_passes, ctx->passes_cap, (size_t)n_int));
    HIP_TRY(ctx, grow(ctx->d_done, ctx->done_cap, (size_t)n_int));
    HIP_TRY(ctx, grow(ctx->d_active, ctx->active_cap, 1));
    HIP_TRY(ctx, grow(ctx->d_dv, ctx->dv_cap, (size_t)n_int * vis->n_ant * ng * 2));
    P.state.dv = ctx->d_dv;
    P.n_part = parts;
    P.partials = ctx->d_partials;
    P.state.passes = ctx->d_passes;
    P.state.done = ctx->d_done;
    P.state.n_active = ctx->d_active;
    P.state.lm = nullptr;
    P.state.acc = nullptr;
    if (lm) {
      HIP_TRY(ctx, grow(ctx->d_lm, ctx->lm_cap, (size_t)n_int * LM_STATE));
      HIP_TRY(ctx, grow(ctx->d_acc, ctx->acc_cap, (size_t)n_int * vis->n_ant * ng * 4));
      P.state.lm = ctx->d_lm;
      P.state.acc = ctx->d_acc;
    }
  }
  size_t dd_off[BAND_MAX_DD] = {0, 0};
  if (band) HIP_TRY(ctx, grow(ctx->d_band, ctx->band_cap, (size_t)std::max<long long>(vis->n_row, 1)));
  if (L.n_dd > 0) {
    size_t dd_bytes = 0;
    for (int j = 0; j < L.n_dd; ++j) {
      dd_off[j] = dd_bytes;
      dd_bytes += (dd_table_bytes(L, L.dd_term[j]) + 255) / 256 * 256;
    }
    HIP_TRY(ctx, grow(ctx->d_ddtab, ctx->ddtab_cap, dd_bytes));
  }
  size_t lds = 0;
  hipError_t e = hipSuccess;
  HIP_TRY(ctx, hipEventRecord(ctx->ev0, s));
  if (want_tab) {
    e = launch_chain_table(L, ctx->d_otab, s);
    L.otab = ctx->d_otab;
  }
  if (band && e == hipSuccess) {
    e = launch_band_steps(L, parts, L.band_rows, ctx->d_band, s);
    L.band_steps = ctx->d_band;
  }
  for (int j = 0; j < L.n_dd && e == hipSuccess; ++j) {
    L.dd_tab[j] = ctx->d_ddtab + dd_off[j];
    e = launch_dd_table(L, L.dd_term[j], ctx->d_ddtab + dd_off[j], s);
  }
  if (e != hipSuccess) {
    // reported below
  } else if (parts <= 1) {
    e = launch_solve(L, nullptr, s, &lds);
  } else {
    P.phase = 0;
    e = launch_solve(L, &P, s, &lds);
    P.phase = 1;
    // a pass per update; with LM a rejected attempt takes one more pass
    const int max_rounds = lm ? 2 * opts->max_iter + 2 : opts->max_iter + 1;
    for (int k = 0; k < max_rounds && e == hipSuccess; ++k) {
      e = launch_solve(L, &P, s, &lds);
      if (e != hipSuccess) break;
      int n_active = 0;
      HIP_TRY(ctx, hipMemcpyAsync(&n_active, ctx->d_active, sizeof(int), hipMemcpyDeviceToHost, s));
      HIP_TRY(ctx, hipStreamSynchronize(s));
      if (n_active <= 0) break;
    }
  }
  if (e != hipSuccess) {
    ctx->timed = false;
    if (lds > 160 * 1024)
      return fail(ctx, QC_E_UNSUPPORTED, "per-interval state needs %zu B of LDS (n_ant=%d)", lds, vis->n_ant);
    return fail(ctx, QC_E_DEVICE, "solve launch: %s", hipGetErrorString(e));
  }
  HIP_TRY(ctx, hipEventRecord(ctx->ev1, s));
  ctx->timed = true;
  return QC_OK;
}

extern "C" {

qc_status qc_solve_interval(qc_ctx* ctx, const qc_vis* vis, qc_term* chain, int32_t n_term, int32_t active,
                            const qc_solve_opts* opts, qc_solve_stats* stats) {
  return solve_interval_impl(ctx, vis, chain, n_term, active, opts, stats, nullptr);
}

qc_status qc_solve_interval_sky(qc_ctx* ctx, const qc_vis* vis, const qc_sky* sky, const double* uvw,
                                qc_term* chain, int32_t n_term, int32_t active, const qc_solve_opts* opts,
                                qc_solve_stats* stats) {
  if (!ctx) return QC_E_ARG;
  if (!sky) return fail(ctx, QC_E_ARG, "sky is NULL");
  return solve_interval_impl(ctx, vis, chain, n_term, active, opts, stats, nullptr, sky, uvw);
}

qc_status qc_solve_interval_static(qc_ctx* ctx, const qc_vis* vis, qc_term* chain, int32_t n_term,
                                   int32_t active, const qc_solve_opts* opts, qc_solve_stats* stats) {
  if (!ctx) return QC_E_ARG;
  if (!chain || n_term <= 0 || active < 0 || active >= n_term)
    return fail(ctx, QC_E_ARG, "active=%d outside the chain of %d terms", active, n_term);
  if (!ctx->static_scratch) return fail(ctx, QC_E_DEVICE, "no scratch array on device %d", ctx->device);
  PrepScratch sc;
  const size_t need = carve_static(ctx->static_scratch, vis, chain[active], sc);
  if (need > QC_STATIC_SCRATCH_BYTES)
    return fail(ctx, QC_E_UNSUPPORTED, "the allocation-free solve needs %zu B of scratch, more than its %d B",
                need, (int)QC_STATIC_SCRATCH_BYTES);
  return solve_interval_impl(ctx, vis, chain, n_term, active, opts, stats, &sc);
}

int32_t qc_ctx_last_split(const qc_ctx* ctx) { return ctx ? ctx->last_split_parts : -1; }

qc_status qc_ctx_set_split(qc_ctx* ctx, int32_t parts) {
  if (!ctx) return QC_E_ARG;
  if (parts < 0) return fail(ctx, QC_E_ARG, "parts must be >= 0");
  ctx->split_parts = parts;
  return QC_OK;
}

qc_status qc_ctx_set_tile(qc_ctx* ctx, int32_t waves, int32_t rows_per_step) {
  if (!ctx) return QC_E_ARG;
  if (waves != 0 && waves != 1 && waves != 2 && waves != 4 && waves != 8)
    return fail(ctx, QC_E_ARG, "waves must be 1, 2, 4 or 8 (0 = default)");
  if (rows_per_step != 0 && rows_per_step != 1 && rows_per_step != 2 && rows_per_step != 4 && rows_per_step != 8)
    return fail(ctx, QC_E_ARG, "rows_per_step must be 1, 2, 4 or 8 (0 = from the interval width)");
  ctx->waves = waves ? waves : 4;
  ctx->rows_per_step = rows_per_step;
  return QC_OK;
}

qc_status qc_solve_chain(qc_ctx* ctx, const qc_vis* vis, qc_term* chain, int32_t n_term, int32_t n_epoch,
                         const qc_solve_opts* opts, qc_solve_stats* stats) {
  if (!ctx) return QC_E_ARG;
  if (n_epoch < 0) return fail(ctx, QC_E_ARG, "n_epoch < 0");
  for (int e = 0; e < n_epoch; ++e) {
    for (int n = 0; n < n_term; ++n) {
      qc_solve_stats* st = stats ? &stats[(size_t)e * n_term + n] : nullptr;
      qc_status s = qc_solve_interval(ctx, vis, chain, n_term, n, opts, st);
      if (s != QC_OK) return s;
    }
  }
  return QC_OK;
}

qc_status qc_solve_chain_robust(qc_ctx* ctx, const qc_vis* vis, qc_term* chain, int32_t n_term, int32_t n_epoch,
                                const qc_solve_opts* opts, double nu, void* resid_work, void* weight_work,
                                qc_solve_stats* stats) {
  if (!ctx) return QC_E_ARG;
  if (!vis || !opts) return fail(ctx, QC_E_ARG, "vis or opts is NULL");
  if (n_epoch < 0) return fail(ctx, QC_E_ARG, "n_epoch < 0");
  if (!(nu > 0.0) || !std::isfinite(nu)) return fail(ctx, QC_E_ARG, "nu must be finite and > 0");
  if (n_epoch > 1 && vis->n_row > 0 && (!resid_work || !weight_work))
    return fail(ctx, QC_E_ARG, "resid_work or weight_work is NULL");
  qc_vis wv = *vis;                            // the weights of the current epoch
  for (int e = 0; e < n_epoch; ++e) {
    for (int n = 0; n < n_term; ++n) {
      qc_solve_stats* st = stats ? &stats[(size_t)e * n_term + n] : nullptr;
      qc_status s = qc_solve_interval(ctx, &wv, chain, n_term, n, opts, st);
      if (s != QC_OK) return s;
    }
    if (e + 1 < n_epoch) {
      // the residual of the whole chain, then weights from the prior ones
      qc_status s = qc_residual(ctx, vis, chain, n_term, nullptr, resid_work, opts->stream);
      if (s != QC_OK) return s;
      s = qc_robust_weights(ctx, vis, resid_work, nu, weight_work, nullptr, opts->stream);
      if (s != QC_OK) return s;
      wv.weight = weight_work;
    }
  }
  return QC_OK;
}

qc_status qc_delay_init(qc_ctx* ctx, const qc_vis* vis, qc_term* k_term, int32_t ref_ant, void* stream) {
  if (!ctx) return QC_E_ARG;
  if (!k_term) return fail(ctx, QC_E_ARG, "term is NULL");
  if (k_term->type != QC_TERM_DELAY && k_term->type != QC_TERM_DELAY_OFFSET)
    return fail(ctx, QC_E_ARG, "qc_delay_init needs a DELAY or DELAY_OFFSET term");
  if (!vis) return fail(ctx, QC_E_ARG, "vis is NULL");
  if (ref_ant < 0 || ref_ant >= vis->n_ant) return fail(ctx, QC_E_ARG, "ref_ant=%d outside [0,%d)", ref_ant, vis->n_ant);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  ctx->last_stream = s;
  std::vector<HostMaps> maps;
  qc_status st = prepare(ctx, vis, k_term, 1, 0, maps, s);
  if (st != QC_OK) return st;
  DelayInitLaunch L;
  memset(&L, 0, sizeof L);
  ChainArgs ca;
  fill_args(vis, k_term, 1, 0, L.vis, ca);
  L.vis_is_c128 = vis->dtype == QC_C128;
  L.offset = k_term->type == QC_TERM_DELAY_OFFSET ? 1 : 0;
  L.n_gt = k_term->n_gt;
  L.n_gf = k_term->n_gf;
  L.n_gdir = k_term->n_gdir;
  L.ref_ant = ref_ant;
  L.row_lo = ctx->d_rowlo;
  L.row_hi = ctx->d_rowhi;
  L.chan_lo = ctx->d_chlo;
  L.chan_hi = ctx->d_chhi;
  L.params = k_term->params;
  L.max_chan = ctx->max_int_chan;
  L.fft = delay_init_lds(L.max_chan, true) <= 64 * 1024;     // up to 1024 channels per interval
  if (delay_init_lds(L.max_chan, L.fft != 0) > 64 * 1024)
    return fail(ctx, QC_E_UNSUPPORTED, "delay interval of %d channels exceeds the LDS budget", ctx->max_int_chan);
  HIP_TRY(ctx, launch_delay_init(L, s));
  return QC_OK;
}

qc_status qc_ws_features(qc_ctx* ctx, const qc_vis* vis, const qc_term* layout, float* feat, double* chisq_unit,
                         int32_t ref_ant, void* stream) {
  if (!ctx) return QC_E_ARG;
  if (!layout || !feat) return fail(ctx, QC_E_ARG, "layout or feat is NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  ctx->last_stream = s;
  std::vector<HostMaps> maps;
  qc_status st = prepare(ctx, vis, layout, 1, 0, maps, s);
  if (st != QC_OK) return st;
  FeatLaunch L;
  memset(&L, 0, sizeof L);
  ChainArgs ca;
  fill_args(vis, layout, 1, 0, L.vis, ca);
  L.vis_is_c128 = vis->dtype == QC_C128;
  L.n_gt = layout->n_gt;
  L.n_gf = layout->n_gf;
  L.row_lo = ctx->d_rowlo;
  L.row_hi = ctx->d_rowhi;
  L.chan_lo = ctx->d_chlo;
  L.chan_hi = ctx->d_chhi;
  L.feat = feat;
  L.feat_stride = vis->n_ant * 8;
  L.chisq_unit = chisq_unit;
  if (ref_ant >= vis->n_ant) return fail(ctx, QC_E_ARG, "ref_ant=%d outside [0,%d)", ref_ant, vis->n_ant);
  L.ref_ant = ref_ant;
  hipError_t e = launch_ws_features(L, 4, s);
  if (e == hipErrorInvalidValue) return fail(ctx, QC_E_UNSUPPORTED, "too many antennas for the feature pass");
  HIP_TRY(ctx, e);
  return QC_OK;
}

static qc_status check_mlp(qc_ctx* ctx, int batch, int n_in, int n_hid, int n_out) {
  if (batch <= 0 || n_in <= 0 || n_hid <= 0 || n_out <= 0)
    return fail(ctx, QC_E_ARG, "bad MLP shape batch=%d in=%d hid=%d out=%d", batch, n_in, n_hid, n_out);
  return QC_OK;
}

qc_status qc_mlp_forward(qc_ctx* ctx, const float* params, const float* x, int32_t batch, int32_t n_in,
                         int32_t n_hid, int32_t n_out, float* y, float* pre, void* stream) {
  if (!ctx) return QC_E_ARG;
  if (!params || !x || !y || !pre) return fail(ctx, QC_E_ARG, "a pointer is NULL");
  qc_status st = check_mlp(ctx, batch, n_in, n_hid, n_out);
  if (st != QC_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  ctx->last_stream = s;
  const float* W1 = params;
  const float* b1 = W1 + (size_t)n_hid * n_in;
  const float* W2 = b1 + n_hid;
  const float* b2 = W2 + (size_t)n_out * n_hid;
  HIP_TRY(ctx, launch_linear_fwd(x, W1, b1, pre, batch, n_in, n_hid, 0, s));
  HIP_TRY(ctx, launch_linear_fwd(pre, W2, b2, y, batch, n_hid, n_out, 1, s));
  return QC_OK;
}

qc_status qc_mlp_backward(qc_ctx* ctx, const float* params, const float* x, const float* pre, const float* dy,
                          int32_t batch, int32_t n_in, int32_t n_hid, int32_t n_out, float* grad, void* stream) {
  if (!ctx) return QC_E_ARG;
  if (!params || !x || !pre || !dy || !grad) return fail(ctx, QC_E_ARG, "a pointer is NULL");
  qc_status st = check_mlp(ctx, batch, n_in, n_hid, n_out);
  if (st != QC_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  ctx->last_stream = s;
  HIP_TRY(ctx, grow(ctx->d_dh, ctx->dh_cap, (size_t)batch * n_hid));
  const float* W2 = params + (size_t)n_hid * n_in + n_hid;
  float* gW1 = grad;
  float* gb1 = gW1 + (size_t)n_hid * n_in;
  float* gW2 = gb1 + n_hid;
  float* gb2 = gW2 + (size_t)n_out * n_hid;
  HIP_TRY(ctx, launch_linear_bwd_w(pre, dy, gW2, gb2, batch, n_hid, n_out, 1, s));
  HIP_TRY(ctx, launch_linear_bwd_x(dy, W2, pre, ctx->d_dh, batch, n_hid, n_out, 1, s));
  HIP_TRY(ctx, launch_linear_bwd_w(x, ctx->d_dh, gW1, gb1, batch, n_in, n_hid, 0, s));
  return QC_OK;
}

qc_status qc_adam_step(qc_ctx* ctx, float* params, const float* grad, float* m, float* v, int32_t n, float lr,
                       float b1, float b2, float eps, int32_t step, void* stream) {
  if (!ctx) return QC_E_ARG;
  if (!params || !grad || !m || !v || n <= 0 || step <= 0) return fail(ctx, QC_E_ARG, "bad Adam arguments");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  ctx->last_stream = s;
  HIP_TRY(ctx, launch_adam(params, grad, m, v, n, lr, b1, b2, eps, step, s));
  return QC_OK;
}

qc_status qc_mse_grad(qc_ctx* ctx, const float* y, const float* t, int32_t n, float* dy, float* loss, void* stream) {
  if (!ctx) return QC_E_ARG;
  if (!y || !t || !dy || n <= 0) return fail(ctx, QC_E_ARG, "bad MSE arguments");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  ctx->last_stream = s;
  HIP_TRY(ctx, launch_mse(y, t, dy, loss, n, s));
  return QC_OK;
}

qc_status qc_ws_gains(qc_ctx* ctx, const float* y, int32_t n_int, int32_t n_ant, void* gains, void* stream) {
  if (!ctx) return QC_E_ARG;
  if (!y || !gains || n_int < 0 || n_ant <= 0) return fail(ctx, QC_E_ARG, "bad warm-start gain arguments");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  ctx->last_stream = s;
  HIP_TRY(ctx, launch_ws_gains(y, n_ant * 4, n_int, n_ant, reinterpret_cast<double2*>(gains), s));
  return QC_OK;
}

qc_status qc_ws_labels(qc_ctx* ctx, const void* gains, int32_t n_int, int32_t n_ant, int32_t ref_ant, float* y,
                       void* stream) {
  if (!ctx) return QC_E_ARG;
  if (!gains || !y || n_int < 0 || n_ant <= 0 || ref_ant < 0 || ref_ant >= n_ant)
    return fail(ctx, QC_E_ARG, "bad warm-start label arguments");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  ctx->last_stream = s;
  HIP_TRY(ctx, launch_ws_labels(reinterpret_cast<const double2*>(gains), n_int, n_ant, ref_ant, y, s));
  return QC_OK;
}

static qc_status outputs_common(qc_ctx* ctx, const qc_vis* vis, const qc_term* chain, int32_t n_term, int mode,
                                const uint8_t* dir_mask, void* out, void* stream, const qc_sky* sky = nullptr,
                                const double* uvw = nullptr) {
  if (!ctx) return QC_E_ARG;
  if (!out) return fail(ctx, QC_E_ARG, "out is NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  ctx->last_stream = s;
  if (sky && !uvw && vis && vis->n_row > 0) return fail(ctx, QC_E_ARG, "uvw is NULL");
  std::vector<HostMaps> maps;
  qc_status st = prepare(ctx, vis, chain, n_term, -1, maps, s, nullptr, sky == nullptr);
  if (st != QC_OK) return st;
  SkyArgs sk;
  memset(&sk, 0, sizeof sk);
  if (sky) {
    st = prepare_sky(ctx, sky, vis->n_dir, uvw, s, sk);
    if (st != QC_OK) return st;
  }
  if (mode == 1 || mode == 3) {
    for (int j = 0; j < n_term; ++j)
      if (!dmap_constant(maps[j]) || chain[j].type == QC_TERM_POINTING)
        return fail(ctx, QC_E_ARG, "%s needs a direction-independent chain (term %d)",
                    mode == 1 ? "CORRECT" : "corrected weights", j);
  }
  OutputLaunch L;
  memset(&L, 0, sizeof L);
  fill_args(vis, chain, n_term, 0, L.vis, L.chain);
  L.vis_is_c128 = vis->dtype == QC_C128;
  L.mode = mode;
  L.diag_chain = 1;
  for (int j = 0; j < n_term; ++j)
    if (chain[j].type == QC_TERM_COMPLEX2X2) L.diag_chain = 0;
  unsigned mask = 0;
  for (int d = 0; d < vis->n_dir; ++d)
    if (!dir_mask || dir_mask[d]) mask |= 1u << d;
  L.dir_mask = mask;
  L.out = out;
  L.w_vec = mode == 3 && vis->n_wcorr == 4 && reinterpret_cast<uintptr_t>(vis->weight) % 16 == 0 &&
            reinterpret_cast<uintptr_t>(out) % 16 == 0;
  L.sky = sk;
  HIP_TRY(ctx, hipEventRecord(ctx->ev0, s));
  HIP_TRY(ctx, launch_outputs(L, s));
  HIP_TRY(ctx, hipEventRecord(ctx->ev1, s));
  ctx->timed = true;
  return QC_OK;
}

qc_status qc_apply_gains(qc_ctx* ctx, const qc_vis* vis, const qc_term* chain, int32_t n_term,
                         qc_apply_mode mode, const uint8_t* dir_mask, void* out, void* stream) {
  const int mode_v = enum_value(mode);
  if (mode_v != QC_CORRUPT && mode_v != QC_CORRECT) return fail(ctx, QC_E_ARG, "bad apply mode %d", mode_v);
  return outputs_common(ctx, vis, chain, n_term, mode == QC_CORRECT ? 1 : 0, dir_mask, out, stream);
}

qc_status qc_residual(qc_ctx* ctx, const qc_vis* vis, const qc_term* chain, int32_t n_term,
                      const uint8_t* dir_mask, void* out, void* stream) {
  return outputs_common(ctx, vis, chain, n_term, 2, dir_mask, out, stream);
}

qc_status qc_corrected_weights(qc_ctx* ctx, const qc_vis* vis, const qc_term* chain, int32_t n_term,
                               void* weight_out, void* stream) {
  return outputs_common(ctx, vis, chain, n_term, 3, nullptr, weight_out, stream);
}

qc_status qc_residual_sky(qc_ctx* ctx, const qc_vis* vis, const qc_sky* sky, const double* uvw,
                          const qc_term* chain, int32_t n_term, const uint8_t* dir_mask, void* out, void* stream) {
  if (!ctx) return QC_E_ARG;
  if (!sky) return fail(ctx, QC_E_ARG, "sky is NULL");
  return outputs_common(ctx, vis, chain, n_term, 2, dir_mask, out, stream, sky, uvw);
}

qc_status qc_corrupt_sky(qc_ctx* ctx, const qc_vis* vis, const qc_sky* sky, const double* uvw,
                         const qc_term* chain, int32_t n_term, const uint8_t* dir_mask, void* out, void* stream) {
  if (!ctx) return QC_E_ARG;
  if (!sky) return fail(ctx, QC_E_ARG, "sky is NULL");
  return outputs_common(ctx, vis, chain, n_term, 0, dir_mask, out, stream, sky, uvw);
}

}  // extern "C"

// Host-side argument checks (see qc_hostcheck.h).

#include "qc_hostcheck.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>

namespace qc {
namespace {

Check bad(qc_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  Check c;
  c.st = st;
  c.msg = buf;
  return c;
}

}  // namespace

Check check_vis_fields(const qc_vis* v, bool need_model) {
  if (!v) return bad(QC_E_ARG, "vis is NULL");
  if (v->n_row < 0 || v->n_chan <= 0 || v->n_dir <= 0 || v->n_ant <= 0 || v->n_time <= 0)
    return bad(QC_E_ARG, "bad sizes: n_row=%lld n_chan=%d n_dir=%d n_ant=%d n_time=%d", (long long)v->n_row,
               v->n_chan, v->n_dir, v->n_ant, v->n_time);
  if (v->n_dir > QC_MAX_DIR) return bad(QC_E_UNSUPPORTED, "n_dir=%d exceeds %d", v->n_dir, QC_MAX_DIR);
  if (v->n_ant > QC_MAX_ANT) return bad(QC_E_UNSUPPORTED, "n_ant=%d exceeds %d", v->n_ant, QC_MAX_ANT);
  if (v->n_wcorr != 1 && v->n_wcorr != 4) return bad(QC_E_ARG, "n_wcorr must be 1 or 4, got %d", v->n_wcorr);
  const int dt = enum_value(v->dtype);
  if (dt != QC_C64 && dt != QC_C128) return bad(QC_E_ARG, "bad dtype %d", dt);
  if (v->n_row > 0 && (!v->data || (need_model && !v->model) || !v->weight || !v->flag || !v->ant1 || !v->ant2 ||
                       !v->row_time))
    return bad(QC_E_ARG, "a visibility array pointer is NULL");
  if (!v->chan_freq) return bad(QC_E_ARG, "chan_freq is NULL");
  return Check{};
}

Check check_term_fields(const qc_term* t, int j) {
  if (!t) return bad(QC_E_ARG, "term %d is NULL", j);
  const int ty = enum_value(t->type);
  if (ty < QC_TERM_DIAGONAL || ty > QC_TERM_POINTING) return bad(QC_E_ARG, "term %d: bad type %d", j, ty);
  if (ty == QC_TERM_POINTING) {
    if (t->n_gdir != 1) return bad(QC_E_ARG, "term %d: a pointing term has n_gdir = 1", j);
    if (!t->dir_lm) return bad(QC_E_ARG, "term %d: dir_lm is NULL", j);
    if (!(std::isfinite(t->beam_fwhm) && t->beam_fwhm > 0.0 && std::isfinite(t->beam_freq) && t->beam_freq > 0.0))
      return bad(QC_E_ARG, "term %d: beam_fwhm and beam_freq must be positive", j);
  }
  if (t->n_gt <= 0 || t->n_gf <= 0 || t->n_gdir <= 0)
    return bad(QC_E_ARG, "term %d: bad gain shape (%d, %d, %d)", j, t->n_gt, t->n_gf, t->n_gdir);
  if (t->n_gdir > QC_MAX_GDIR) return bad(QC_E_UNSUPPORTED, "term %d: n_gdir=%d exceeds %d", j, t->n_gdir, QC_MAX_GDIR);
  if (!t->t_map || !t->f_map || !t->d_map) return bad(QC_E_ARG, "term %d: a map pointer is NULL", j);
  const bool real_params = ty >= QC_TERM_DELAY;   // delay, phase, amplitude, delay and offset, pointing
  if (real_params ? !t->params : !t->gains)
    return bad(QC_E_ARG, "term %d: %s is NULL", j, real_params ? "params" : "gains");
  return Check{};
}

Check check_dir_lm(const double* lm, int n_dir, int j) {
  for (int i = 0; i < 2 * n_dir; ++i)
    if (!std::isfinite(lm[i])) return bad(QC_E_ARG, "term %d: non-finite dir_lm", j);
  return Check{};
}

Check check_term_maps(const qc_term* t, int j, const int* t_map, int n_time, const int* f_map, int n_chan,
                      const int* d_map, int n_dir) {
  for (int i = 0; i < n_time; ++i) {
    if (t_map[i] < 0 || t_map[i] >= t->n_gt)
      return bad(QC_E_RANGE, "term %d: t_map[%d]=%d outside [0,%d)", j, i, t_map[i], t->n_gt);
    if (i > 0 && t_map[i] < t_map[i - 1]) return bad(QC_E_ARG, "term %d: t_map is not non-decreasing at %d", j, i);
  }
  for (int i = 0; i < n_chan; ++i) {
    if (f_map[i] < 0 || f_map[i] >= t->n_gf)
      return bad(QC_E_RANGE, "term %d: f_map[%d]=%d outside [0,%d)", j, i, f_map[i], t->n_gf);
    if (i > 0 && f_map[i] < f_map[i - 1]) return bad(QC_E_ARG, "term %d: f_map is not non-decreasing at %d", j, i);
  }
  for (int i = 0; i < n_dir; ++i)
    if (d_map[i] < 0 || d_map[i] >= t->n_gdir)
      return bad(QC_E_RANGE, "term %d: d_map[%d]=%d outside [0,%d)", j, i, d_map[i], t->n_gdir);
  return Check{};
}

int interval_extents(const std::vector<int>& t_map, const std::vector<int>& f_map, int n_gt, int n_gf,
                     std::vector<int>& tt, std::vector<int>& clo, std::vector<int>& chi) {
  tt.assign(2 * (size_t)std::max(n_gt, 0), 0);
  clo.assign((size_t)std::max(n_gf, 0), 0);
  chi.assign((size_t)std::max(n_gf, 0), 0);
  int widest = 0;
  for (int g = 0; g < n_gt; ++g) {
    tt[g] = (int)(std::lower_bound(t_map.begin(), t_map.end(), g) - t_map.begin());
    tt[n_gt + g] = (int)(std::upper_bound(t_map.begin(), t_map.end(), g) - t_map.begin());
  }
  for (int g = 0; g < n_gf; ++g) {
    clo[g] = (int)(std::lower_bound(f_map.begin(), f_map.end(), g) - f_map.begin());
    chi[g] = (int)(std::upper_bound(f_map.begin(), f_map.end(), g) - f_map.begin());
    widest = std::max(widest, chi[g] - clo[g]);
  }
  return widest;
}

}  // namespace qc

// Driver of the C-ABI's host argument checks (csrc/qc_hostcheck.cpp) for a
// build under the host address and undefined-behaviour sanitizers
// (test_host_sanitize.py): malformed and edge-case visibility sets, terms
// and maps with the status each must give, and interval extents against a
// brute-force count on random maps.  Exit status 0 when every case agrees.
#include <climits>
#include <cmath>
#include <cstdio>
#include <limits>
#include <random>
#include <vector>

#include "../paper_2412_10072_amd/csrc/qc_hostcheck.h"

static int failures = 0;
static int cases = 0;

static void expect(const char* what, const qc::Check& c, qc_status want) {
  ++cases;
  if (c.st != want) {
    std::printf("FAIL %s: status %d, expected %d (%s)\n", what, (int)c.st, (int)want, c.msg.c_str());
    ++failures;
  } else if ((want == QC_OK) != c.msg.empty()) {
    std::printf("FAIL %s: message '%s' with status %d\n", what, c.msg.c_str(), (int)c.st);
    ++failures;
  }
}

// host stand-ins for the arrays: the checks read only the pointers' nullness
static const double kDummy[4] = {0, 0, 0, 0};
static const int kDummyI[4] = {0, 0, 0, 0};
static const uint8_t kDummyU[4] = {0, 0, 0, 0};

static qc_vis good_vis() {
  qc_vis v{};
  v.n_row = 10;
  v.n_chan = 4;
  v.n_dir = 2;
  v.n_ant = 5;
  v.n_time = 3;
  v.n_wcorr = 4;
  v.dtype = QC_C64;
  v.data = kDummy;
  v.model = kDummy;
  v.weight = kDummy;
  v.flag = kDummyU;
  v.ant1 = kDummyI;
  v.ant2 = kDummyI;
  v.row_time = kDummyI;
  v.chan_freq = kDummy;
  return v;
}

static qc_term good_term(qc_term_type type) {
  qc_term t{};
  t.type = type;
  t.n_gt = 2;
  t.n_gf = 2;
  t.n_gdir = 1;
  t.t_map = kDummyI;
  t.f_map = kDummyI;
  t.d_map = kDummyI;
  t.gains = const_cast<double*>(kDummy);
  t.params = const_cast<double*>(kDummy);
  t.dir_lm = kDummy;
  t.beam_fwhm = 0.02;
  t.beam_freq = 1.4e9;
  return t;
}

static void vis_cases() {
  expect("vis NULL", qc::check_vis_fields(nullptr, true), QC_E_ARG);
  const qc_vis gv = good_vis();
  expect("vis good", qc::check_vis_fields(&gv, true), QC_OK);
  struct Case {
    const char* what;
    void (*edit)(qc_vis&);
    qc_status want;
  };
  const Case cs[] = {
      {"n_row < 0", [](qc_vis& v) { v.n_row = -1; }, QC_E_ARG},
      {"n_row = INT64_MIN", [](qc_vis& v) { v.n_row = LLONG_MIN; }, QC_E_ARG},
      {"n_chan = 0", [](qc_vis& v) { v.n_chan = 0; }, QC_E_ARG},
      {"n_dir = 0", [](qc_vis& v) { v.n_dir = 0; }, QC_E_ARG},
      {"n_ant < 0", [](qc_vis& v) { v.n_ant = INT_MIN; }, QC_E_ARG},
      {"n_time = 0", [](qc_vis& v) { v.n_time = 0; }, QC_E_ARG},
      {"n_dir above the limit", [](qc_vis& v) { v.n_dir = QC_MAX_DIR + 1; }, QC_E_UNSUPPORTED},
      {"n_dir = INT_MAX", [](qc_vis& v) { v.n_dir = INT_MAX; }, QC_E_UNSUPPORTED},
      {"n_ant above the limit", [](qc_vis& v) { v.n_ant = QC_MAX_ANT + 1; }, QC_E_UNSUPPORTED},
      {"n_wcorr = 2", [](qc_vis& v) { v.n_wcorr = 2; }, QC_E_ARG},
      {"n_wcorr = 0", [](qc_vis& v) { v.n_wcorr = 0; }, QC_E_ARG},
      {"n_wcorr = 1", [](qc_vis& v) { v.n_wcorr = 1; }, QC_OK},
      {"dtype 7", [](qc_vis& v) { v.dtype = (qc_dtype)7; }, QC_E_ARG},
      {"dtype -1", [](qc_vis& v) { v.dtype = (qc_dtype)-1; }, QC_E_ARG},
      {"dtype C128", [](qc_vis& v) { v.dtype = QC_C128; }, QC_OK},
      {"data NULL", [](qc_vis& v) { v.data = nullptr; }, QC_E_ARG},
      {"model NULL", [](qc_vis& v) { v.model = nullptr; }, QC_E_ARG},
      {"weight NULL", [](qc_vis& v) { v.weight = nullptr; }, QC_E_ARG},
      {"flag NULL", [](qc_vis& v) { v.flag = nullptr; }, QC_E_ARG},
      {"ant1 NULL", [](qc_vis& v) { v.ant1 = nullptr; }, QC_E_ARG},
      {"ant2 NULL", [](qc_vis& v) { v.ant2 = nullptr; }, QC_E_ARG},
      {"row_time NULL", [](qc_vis& v) { v.row_time = nullptr; }, QC_E_ARG},
      {"chan_freq NULL", [](qc_vis& v) { v.chan_freq = nullptr; }, QC_E_ARG},
      {"no rows, NULL arrays", [](qc_vis& v) {
         v.n_row = 0;
         v.data = v.model = v.weight = nullptr;
         v.flag = nullptr;
         v.ant1 = v.ant2 = v.row_time = nullptr;
       }, QC_OK},
      {"no rows, chan_freq NULL", [](qc_vis& v) { v.n_row = 0; v.chan_freq = nullptr; }, QC_E_ARG},
  };
  for (const Case& c : cs) {
    qc_vis v = good_vis();
    c.edit(v);
    expect(c.what, qc::check_vis_fields(&v, true), c.want);
  }
  qc_vis v = good_vis();
  v.model = nullptr;
  expect("model NULL, predicted model", qc::check_vis_fields(&v, false), QC_OK);
}

static void term_cases() {
  expect("term NULL", qc::check_term_fields(nullptr, 0), QC_E_ARG);
  const qc_term_type types[] = {QC_TERM_DIAGONAL, QC_TERM_COMPLEX2X2, QC_TERM_DELAY, QC_TERM_PHASE,
                                QC_TERM_AMPLITUDE, QC_TERM_DELAY_OFFSET, QC_TERM_POINTING};
  for (qc_term_type ty : types) {
    qc_term t = good_term(ty);
    expect("term good", qc::check_term_fields(&t, 1), QC_OK);
    t.n_gt = 0;
    expect("n_gt = 0", qc::check_term_fields(&t, 1), QC_E_ARG);
    t = good_term(ty);
    t.n_gf = INT_MIN;
    expect("n_gf < 0", qc::check_term_fields(&t, 1), QC_E_ARG);
    t = good_term(ty);
    t.t_map = nullptr;
    expect("t_map NULL", qc::check_term_fields(&t, 1), QC_E_ARG);
    t = good_term(ty);
    t.d_map = nullptr;
    expect("d_map NULL", qc::check_term_fields(&t, 1), QC_E_ARG);
    t = good_term(ty);
    const bool real = ty >= QC_TERM_DELAY;
    if (real) t.params = nullptr;
    else t.gains = nullptr;
    expect("values NULL", qc::check_term_fields(&t, 1), QC_E_ARG);
    t = good_term(ty);
    if (real) t.gains = nullptr;      // the other array is not read
    else t.params = nullptr;
    expect("the other values NULL", qc::check_term_fields(&t, 1), QC_OK);
  }
  qc_term t = good_term(QC_TERM_DIAGONAL);
  t.type = (qc_term_type)7;
  expect("type 7", qc::check_term_fields(&t, 0), QC_E_ARG);
  t.type = (qc_term_type)-1;
  expect("type -1", qc::check_term_fields(&t, 0), QC_E_ARG);
  t = good_term(QC_TERM_DIAGONAL);
  t.n_gdir = QC_MAX_GDIR + 1;
  expect("n_gdir above the limit", qc::check_term_fields(&t, 0), QC_E_UNSUPPORTED);
  t.n_gdir = QC_MAX_GDIR;
  expect("n_gdir at the limit", qc::check_term_fields(&t, 0), QC_OK);
  // pointing
  t = good_term(QC_TERM_POINTING);
  t.n_gdir = 2;
  expect("pointing n_gdir = 2", qc::check_term_fields(&t, 0), QC_E_ARG);
  t = good_term(QC_TERM_POINTING);
  t.dir_lm = nullptr;
  expect("pointing dir_lm NULL", qc::check_term_fields(&t, 0), QC_E_ARG);
  const double nan = std::numeric_limits<double>::quiet_NaN(), inf = std::numeric_limits<double>::infinity();
  const double bad_beam[] = {0.0, -0.02, nan, inf, -inf};
  for (double b : bad_beam) {
    t = good_term(QC_TERM_POINTING);
    t.beam_fwhm = b;
    expect("pointing beam_fwhm", qc::check_term_fields(&t, 0), QC_E_ARG);
    t = good_term(QC_TERM_POINTING);
    t.beam_freq = b;
    expect("pointing beam_freq", qc::check_term_fields(&t, 0), QC_E_ARG);
  }
  const double lm_ok[] = {0.01, -0.02, 0.0, 0.003};
  expect("dir_lm finite", qc::check_dir_lm(lm_ok, 2, 0), QC_OK);
  for (int i = 0; i < 4; ++i) {
    double lm[4] = {0.01, -0.02, 0.0, 0.003};
    lm[i] = (i & 1) ? inf : nan;
    expect("dir_lm non-finite", qc::check_dir_lm(lm, 2, 0), QC_E_ARG);
  }
  expect("dir_lm no directions", qc::check_dir_lm(nullptr, 0, 0), QC_OK);
}

static void map_cases() {
  qc_term t = good_term(QC_TERM_DIAGONAL);
  t.n_gt = 3;
  t.n_gf = 2;
  t.n_gdir = 2;
  std::vector<int> tm = {0, 0, 1, 2, 2}, fm = {0, 0, 1, 1}, dm = {0, 1, 1};
  auto run = [&](const char* what, qc_status want) {
    expect(what, qc::check_term_maps(&t, 0, tm.data(), (int)tm.size(), fm.data(), (int)fm.size(), dm.data(),
                                     (int)dm.size()), want);
  };
  run("maps good", QC_OK);
  tm[0] = -1;
  run("t_map negative", QC_E_RANGE);
  tm[0] = 0;
  tm[4] = 3;
  run("t_map = n_gt", QC_E_RANGE);
  tm[4] = INT_MAX;
  run("t_map = INT_MAX", QC_E_RANGE);
  tm[4] = 2;
  tm[2] = 0;
  tm[3] = 2;
  tm[1] = 1;
  run("t_map decreasing", QC_E_ARG);
  tm = {0, 0, 1, 2, 2};
  fm[3] = 0;
  run("f_map decreasing", QC_E_ARG);
  fm[3] = 2;
  run("f_map = n_gf", QC_E_RANGE);
  fm[3] = INT_MIN;
  run("f_map = INT_MIN", QC_E_RANGE);
  fm = {0, 0, 1, 1};
  dm[2] = 2;
  run("d_map = n_gdir", QC_E_RANGE);
  dm[2] = -1;
  run("d_map negative", QC_E_RANGE);
  dm = {1, 0, 1};
  run("d_map in any order", QC_OK);
  tm = {2, 2, 2, 2, 2};
  dm = {0, 1, 1};
  run("every time in the last gain time", QC_OK);
}

// interval extents against a count over the maps
static void extent_cases() {
  std::mt19937 rng(2412);
  for (int trial = 0; trial < 2000; ++trial) {
    const int n_time = 1 + (int)(rng() % 40), n_chan = 1 + (int)(rng() % 70);
    const int n_gt = 1 + (int)(rng() % 12), n_gf = 1 + (int)(rng() % 12);
    std::vector<int> tm(n_time), fm(n_chan);
    int g = 0;
    for (int i = 0; i < n_time; ++i) {
      if (rng() % 3 == 0 && g < n_gt - 1) g += 1 + (int)(rng() % (unsigned)(n_gt - 1 - g));
      tm[i] = g;
    }
    g = (int)(rng() % (unsigned)n_gf);
    for (int i = 0; i < n_chan; ++i) {
      if (rng() % 4 == 0 && g < n_gf - 1) ++g;
      fm[i] = g;
    }
    std::vector<int> tt, clo, chi;
    const int widest = qc::interval_extents(tm, fm, n_gt, n_gf, tt, clo, chi);
    ++cases;
    bool ok = (int)tt.size() == 2 * n_gt && (int)clo.size() == n_gf && (int)chi.size() == n_gf;
    int want_widest = 0;
    for (int k = 0; ok && k < n_gt; ++k) {
      int count = 0, first = -1;
      for (int i = 0; i < n_time; ++i)
        if (tm[i] == k) {
          if (first < 0) first = i;
          ++count;
        }
      ok = tt[n_gt + k] - tt[k] == count && (count == 0 || tt[k] == first);
    }
    for (int k = 0; ok && k < n_gf; ++k) {
      int count = 0, first = -1;
      for (int i = 0; i < n_chan; ++i)
        if (fm[i] == k) {
          if (first < 0) first = i;
          ++count;
        }
      ok = chi[k] - clo[k] == count && (count == 0 || clo[k] == first);
      if (count > want_widest) want_widest = count;
    }
    ok = ok && widest == want_widest;
    if (!ok) {
      std::printf("FAIL interval extents, trial %d (n_time %d, n_chan %d, n_gt %d, n_gf %d)\n", trial, n_time,
                  n_chan, n_gt, n_gf);
      ++failures;
      return;
    }
  }
}

int main() {
  vis_cases();
  term_cases();
  map_cases();
  extent_cases();
  std::printf("%d cases, %d failures\n", cases, failures);
  return failures == 0 ? 0 : 1;
}

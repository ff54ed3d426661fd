// Host-side argument checks of the C-ABI that need no device: the fields of a
// visibility set and of a chain term, a term's maps (host copies), a pointing
// term's direction cosines, and the time and channel extent of every solution
// interval (solution intervals as mappings from data to gain indices, Section
// 4.3).  Plain C++ without HIP, so that the same code also builds on its own
// under host sanitizers.
#pragma once

#include <cstring>
#include <string>
#include <vector>

#include "../../include/qc.h"

namespace qc {

// The integer a caller stored in an enum field of an argument struct: the C
// ABI lets a caller store any int there, and in C++ loading an enum object
// that holds a value outside its enumerators' range is undefined, so enum
// arguments are read as their bytes and compared as ints.
template <typename E>
inline int enum_value(const E& e) {
  static_assert(sizeof(E) == sizeof(int), "C enums are int-sized");
  int v;
  std::memcpy(&v, &e, sizeof v);
  return v;
}

struct Check {
  qc_status st = QC_OK;
  std::string msg;           // empty when st == QC_OK
};

// Sizes, limits, enumerations and non-null pointers of a visibility set.
// need_model false: v->model may be NULL (a model predicted from a sky).
Check check_vis_fields(const qc_vis* v, bool need_model);

// Type, gain shape and pointers of chain term j (its maps are checked after
// they are copied to the host: check_term_maps).
Check check_term_fields(const qc_term* t, int j);

// A pointing term's direction cosines [n_dir][2] (host copy): finite.
Check check_dir_lm(const double* lm, int n_dir, int j);

// Term j's maps (host copies): t_map [n_time] into [0, n_gt) and
// non-decreasing, f_map [n_chan] into [0, n_gf) and non-decreasing, d_map
// [n_dir] into [0, n_gdir).
Check check_term_maps(const qc_term* t, int j, const int* t_map, int n_time, const int* f_map, int n_chan,
                      const int* d_map, int n_dir);

// Time range [tt[g], tt[n_gt + g]) of every gain time and channel range
// [clo[g], chi[g]) of every gain frequency of validated maps (a gain index
// that no time or channel maps to gets an empty range); returns the channel
// count of the widest interval.
int interval_extents(const std::vector<int>& t_map, const std::vector<int>& f_map, int n_gt, int n_gf,
                     std::vector<int>& tt, std::vector<int>& clo, std::vector<int>& chi);

}  // namespace qc

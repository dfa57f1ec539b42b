// Internal declarations shared by the host sources of the library (not part of the ABI).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "ch_ib.h"

struct ch_ib_geometry {
  ch_ib_grid grid;
  int ndim = 0;
  int n[3] = {1, 1, 1};
  double lo[3] = {0, 0, 0};
  double h = 0.0;
  int64_t cells = 0;
  int64_t n_ghost = 0;
  int n_ap = 0;
  std::vector<int64_t> gidx;     // [G]
  std::vector<double> normal;    // [d][G]
  std::vector<double> dn;        // [G]
  std::vector<double> gamma;     // [G]
  std::vector<int64_t> ap;       // [2][K][G]
  std::vector<double> w;         // [2][K][G]
  std::vector<double> alpha;     // [cells] or empty
  std::vector<double> face_alpha;   // [ndim][cells] staggered-cell fractions, or empty
};

namespace chib {

void set_error(const std::string &msg);
int fail(int code, const std::string &msg);

// Validates a grid and fills the derived fields of a geometry object (n, lo, h, cells).
int check_grid(const ch_ib_grid *grid, ch_ib_geometry *g);

struct Plan;

// Access to a state's device plan for the other device sources of the library.  state_ref runs
// a pending initial ghost fill first; state_mark_reinit makes the next step start over from the
// current C (C_prev := C, ghosts refilled).
struct StateRef {
  Plan *plan;
  int cur;
  int es;
};
int state_ref(ch_ib_state *st, StateRef *out);
void state_mark_reinit(ch_ib_state *st);
// The momentum step's history flags (first step pending, advecting velocity valid) of `from`
// given to `to` (whose momentum fields were restricted from `from`'s).
void state_copy_momentum_flags(const ch_ib_state *from, ch_ib_state *to);

}  // namespace chib

// Device-resident small state of one GMRES solve.
#pragma once

#include "sa_internal.h"

namespace sa {

constexpr int GMAX = 128;   // largest restart length

struct GTail {
  double bnorm2, bnorm, rnorm2, beta, inv, tol, relres;
  int active, converged, breakdown, nonfinite, have_update;
  int jdone, jlimit;
  long long iters, matvecs;
};

struct GState {
  double H[(GMAX + 1) * GMAX];   // column j at H + j*(GMAX+1)
  double cs[GMAX], sn[GMAX];
  double g[GMAX + 1];
  double y[GMAX];
  double d1[GMAX + 2];           // first CGS pass: V^T w, then ||w||^2 (A z_j, unorthogonalised)
  double d2[GMAX + 1];           // second CGS pass: V^T w
  double wn2;                    // ||w||^2 after both passes
  GTail t;                       // scalars, copied to the host once per cycle
};

void gstate_init(GState* st, double tol, int jlimit, hipStream_t s);
void gstate_set_bnorm(GState* st, hipStream_t s);
void gstate_set_jlimit(GState* st, int jlimit, hipStream_t s);
void gstate_cycle_start(GState* st, hipStream_t s);
void gstate_step(GState* st, int j, hipStream_t s);
void gstate_finish(GState* st, hipStream_t s);

}  // namespace sa

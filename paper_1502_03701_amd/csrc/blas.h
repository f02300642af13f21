// Launchers of the Krylov vector kernels (see blas.hip).
#pragma once

#include "gmres_small.h"
#include "sa_internal.h"

namespace sa {

constexpr int PARTIAL_LD = 160;

// A batch of independent systems handled by one launch: system s uses
// vectors offset by s*vec, device results offset by s*res (doubles), active
// flags offset by s*act (ints).  nsys = 1 with zero strides is a single system.
struct Batch {
  int nsys = 1;
  long long vec = 0;    // stride of the basis / vector arrays (elements)
  long long res = 0;    // stride of device result arrays (doubles)
  long long act = 0;    // stride of the active flags (ints)
  long long wvec = -1;  // stride of the w / wout vectors of update (-1: vec)
  long long w() const { return wvec < 0 ? vec : wvec; }
};

// Reductions over at most this many blocks finish inside the reducing kernel
// (the last block to arrive sums the partials), larger ones in a second kernel.
constexpr int FUSE_MAX_BLOCKS = 256;

// A partial-sum workspace (nsys x RED_BLOCKS x ldp doubles) bound to the
// launchers, and nsys zero-initialised arrival counters (null: reductions
// always finish in a second kernel).
template <typename R>
struct Blas {
  double* partial = nullptr;
  int* ticket = nullptr;
  int ldp = PARTIAL_LD;

  // out[0..ncol) (+)= V^T w, V column c at V + c*ldv.
  void multidot(long long n, const R* V, long long ldv, int ncol, const R* w, double* out, bool accumulate,
                const int* active, hipStream_t s, const Batch& b = Batch()) const;
  // wout = w + hsign * V h; mode 0: nothing else, 1: out (+)= V^T wout,
  // 2: out (+)= ||wout||^2.  wout may alias w.  With mode 2 and a GMRES state
  // array `step` (one per system, stride b.res), the Arnoldi step j of each
  // system follows the norm (gstate_step semantics), fused into the same
  // launch when the reduction is; returns whether it was fused (else the
  // caller launches the step).
  bool update(long long n, const R* V, long long ldv, int ncol, const double* h, double hsign, const R* w,
              R* wout, int mode, double* out, bool accumulate, const int* active, hipStream_t s,
              const Batch& b = Batch(), GState* step = nullptr, int step_j = 0) const;
  void nrm2sq(long long n, const R* x, double* out, const int* active, hipStream_t s,
              const Batch& b = Batch()) const;
  // r = b - y, out = ||r||^2; r uses the batch's vec stride, b and y their own
  void residual(long long n, const R* bvec, const R* y, R* r, double* out, const int* active, hipStream_t s,
                const Batch& b = Batch(), long long sB = 0, long long sY = 0) const;
  // out = x * (*a)
  void scale(long long n, const R* x, R* out, const double* a, const int* active, hipStream_t s,
             const Batch& b = Batch()) const;
  void fill(long long n, R* x, R v, hipStream_t s) const;
  // out = a x + c y for nsys systems (strides sx, sy, so; y may equal x),
  // skipped for systems whose flag active[sys * sA] is 0
  void lincomb(long long n, int nsys, const R* x, long long sx, double a, const R* y, long long sy, double c, R* out,
               long long so, const int* active, long long sA, hipStream_t s) const;
};

// out = float(x * (*scale)) (scale may be null)
void cast_d2f(long long n, const double* x, float* out, const double* scale, hipStream_t s);
// out += double(x) * (*scale)
void axpy_f2d(long long n, const float* x, double* out, const double* scale, hipStream_t s);

}  // namespace sa

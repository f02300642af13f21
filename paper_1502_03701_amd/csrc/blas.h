// Launchers of the Krylov vector kernels (see blas.hip).
#pragma once

#include "sa_internal.h"

namespace sa {

// A partial-sum workspace (RED_BLOCKS x ldp doubles) bound to the launchers.
template <typename R>
struct Blas {
  double* partial = nullptr;
  int ldp = 0;

  // out[0..ncol) (+)= V^T w, V column c at V + c*ldv.
  void multidot(long long n, const R* V, long long ldv, int ncol, const R* w, double* out,
                bool accumulate, const int* active, hipStream_t s) const;
  // wout = w + hsign * V h; mode 0: nothing else, 1: out (+)= V^T wout,
  // 2: out (+)= ||wout||^2.  wout may alias w.
  void update(long long n, const R* V, long long ldv, int ncol, const double* h, double hsign,
              const R* w, R* wout, int mode, double* out, bool accumulate, const int* active,
              hipStream_t s) const;
  void nrm2sq(long long n, const R* x, double* out, const int* active, hipStream_t s) const;
  // r = b - y, out = ||r||^2
  void residual(long long n, const R* b, const R* y, R* r, double* out, const int* active,
                hipStream_t s) const;
  // out = x * (*a)
  void scale(long long n, const R* x, R* out, const double* a, const int* active,
             hipStream_t s) const;
  void fill(long long n, R* x, R v, hipStream_t s) const;
};

// out = float(x * (*scale)) (scale may be null)
void cast_d2f(long long n, const double* x, float* out, const double* scale, hipStream_t s);
// out += double(x) * (*scale)
void axpy_f2d(long long n, const float* x, double* out, const double* scale, hipStream_t s);

constexpr int PARTIAL_LD = 160;

}  // namespace sa

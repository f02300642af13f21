// Internal declarations shared by the HIP translation units of libsa.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

namespace sa {

// Physical and grid parameters of one problem, as the kernels consume them.
struct OpParams {
  int ndim;
  int nx, ny, nz;
  int bcy;                 // 0 periodic, 1 walls at j = 0 and ny-1
  long long npts;
  double ihx, ihy, ihz;    // 1/h
  double gamma;
  double cp;               // c_p = gamma R/(gamma-1)
  double R;                // gas constant, 1/(gamma M^2)
  double p_ref;            // reference pressure, 1/(gamma M^2)
  double mu_ref;           // 1/Re (0 inviscid)
  double suth;             // Sutherland constant S/T_ref
  double pr;
};

// Kernel launchers (all enqueue on the given stream; no synchronisation).
// Jv: y = (J - shift I) x for nrhs vectors.  base holds the nv base fields
// followed by three pointwise fields T0, dT/dp, dT/ds (all with walls).
template <typename R>
hipError_t launch_jv_tiled(const OpParams& p, const R* base, const R* x, R* y, int nrhs, R shift,
                           const int* active, hipStream_t s);
// Reference kernel (one thread per point, stencil taps straight from memory).
template <typename R>
hipError_t launch_jv_direct(const OpParams& p, const R* base, const R* x, R* y, int nrhs, R shift,
                            const int* active, hipStream_t s);
// Operator dispatch: the tiled kernel, or the reference kernel when the
// process was started with SA_JV_REFERENCE=1 (used to cross-check tilings).
template <typename R>
hipError_t launch_jv(const OpParams& p, const R* base, const R* x, R* y, int nrhs, R shift,
                     const int* active, hipStream_t s);

// Base-state preprocessing: fields T0, T_p, T_s appended after q0 (FP64),
// and the FP32 shadow of the whole base array.  Returns via flag (device int)
// nonzero if q0 has NaN/Inf or non-positive pressure.
hipError_t launch_base_derive(const OpParams& p, double* base, float* base32, int* flag,
                              hipStream_t s);

// ----- vector kernels (blas.hip) -----
// Deterministic reductions: each block writes a partial, a second kernel
// sums partials in a fixed order.
constexpr int RED_BLOCKS = 1024;   // partial count used by every reduction
constexpr int RED_THREADS = 256;

}  // namespace sa

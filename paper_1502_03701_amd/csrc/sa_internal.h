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
// Tiled kernel; with bdata (per-point base-state data from launch_base_data,
// base_data_fields(ndim) fields) only the perturbation is differentiated.
template <typename R>
hipError_t launch_jv_tiled(const OpParams& p, const R* base, const R* x, R* y, int nrhs, R shift,
                           const int* active, const R* bdata, hipStream_t s);
int base_data_fields(int ndim);
// Perturbation-only kernels with a register z-queue (need bdata).  nrhs
// systems in one launch: system r uses x/y + r*sV (sV = 0: n), the shift
// shifts[r] (device array; null: the scalar shift) and active[r*sA].
// launch_jv_prefetch (jv_prefetch.hip) prefetches the next plane (16 x 16
// tiles); launch_jv_stage (jv_stage.hip) stages whole planes (32 x 8 tiles);
// nzc (1, 4, 16 or 32) is the number of z planes a workgroup marches over.
template <typename R>
hipError_t launch_jv_prefetch(const OpParams& p, const R* base, const R* bdata, const R* x, R* y, int nrhs, R shift,
                              const int* active, hipStream_t s, long long sX, long long sY, const double* shifts,
                              long long sA, int nzc);
template <typename R>
hipError_t launch_jv_stage(const OpParams& p, const R* base, const R* bdata, const R* x, R* y, int nrhs, R shift,
                           const int* active, hipStream_t s, long long sX, long long sY, const double* shifts,
                           long long sA, int nzc);
// The variants of the perturbation-only kernel (values of sa.h's
// sa_jv_variant); -1 is the precision's default (prefetch z32 in FP64,
// stage z16 in FP32).
// prefetch z32, prefetch z16, stage z16, stage z32, prefetch z4, prefetch z1,
// stage z4, stage z1 (zN: N planes per workgroup; shallow ones give small 3D
// grids enough workgroups)
constexpr int JV_NVARIANTS = 8;
template <typename R>
hipError_t launch_jv_pert(const OpParams& p, const R* base, const R* bdata, const R* x, R* y, int nrhs, R shift,
                          const int* active, hipStream_t s, long long sX = 0, long long sY = 0,
                          const double* shifts = nullptr, long long sA = 0, int variant = -1);
// A batch of systems: one launch with the default kernel, else one launch per
// system.  System r reads x + r*sX, writes y + r*sY; shifts_host / shifts_dev
// hold the per-system shifts.
template <typename R>
hipError_t launch_jv_batch(const OpParams& p, const R* base, const R* bdata, const R* x, R* y, int nsys,
                           long long sX, long long sY, const double* shifts_host, const double* shifts_dev,
                           const int* active, long long sA, hipStream_t s, int variant = -1);
hipError_t launch_base_data(const OpParams& p, const double* base, double* bdata, hipStream_t s);
// Reference kernel (one thread per point, stencil taps straight from memory).
template <typename R>
hipError_t launch_jv_direct(const OpParams& p, const R* base, const R* x, R* y, int nrhs, R shift,
                            const int* active, hipStream_t s);
// Operator dispatch: the perturbation-only kernel variant given (-1: the
// precision's default), one of them for both precisions
// (SA_JV_KERNEL=prefetch or stage), the tiled
// kernel with precomputed base data (SA_JV_KERNEL=tiled), the tiled kernel
// differentiating the base state every call (SA_JV_KERNEL=onthefly) or the
// reference kernel (SA_JV_KERNEL=reference); the variable is read once per
// process and serves to cross-check kernels.
template <typename R>
hipError_t launch_jv(const OpParams& p, const R* base, const R* bdata, const R* x, R* y, int nrhs, R shift,
                     const int* active, hipStream_t s, int variant = -1);
// Whether SA_JV_KERNEL forces a kernel (then variants are not tuned).
bool jv_kernel_forced();

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

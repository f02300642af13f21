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
  // IsoBase<double> / IsoBase<float> (host memory of the context) when the
  // base state has a uniform thermodynamic state, else null
  const void* iso[2];
  // first derivatives: 0 explicit differences, 1 compact (compact.hip), with
  // its workspace (compact_work_elems doubles, one system at a time) and
  // Thomas tables (compact_table_elems, double and float)
  int scheme;
  void* cwork;
  const double* ctab64;
  const float* ctab32;
  // y metric per row j (device, [3][ny]): m1 = 1/h_y, m2 = 1/h_y^2 and
  // m4 = 0 on a uniform grid; with the stretched rows y(eta) the scales
  // 1/(h_eta y'), 1/(h_eta y')^2 and -y''/y'^2, so that D_y f = m1 d1 f and
  // D_yy f = m2 d2 f + m4 D_y f (d1, d2: the stencil sums along the rows)
  const double* ym64;
  const float* ym32;
  double stretch;          // beta (0: uniform rows)
};
template <typename R>
__device__ __forceinline__ const R* ymet(const OpParams& op);
template <>
__device__ __forceinline__ const double* ymet<double>(const OpParams& op) {
  return op.ym64;
}
template <>
__device__ __forceinline__ const float* ymet<float>(const OpParams& op) {
  return op.ym32;
}

// Base states with uniform p0 and s0 (so uniform T0, rho0, mu0, dT/dp,
// dT/ds): the operator needs per point only u0_i, D_a u0_i and
// L u0_i + G0_i/3 (iso_fields(ND) fields, in that order, D_a u0_i at
// ND + i ND + a), each classified exactly as identically zero, a y profile
// (equal along x and z; read at x = 0, z = 0) or general.
constexpr int ISO_MAXF = 15;
__host__ __device__ constexpr int iso_fields(int nd) { return nd + nd * nd + nd; }
// base-data field holding iso field q: u0_i at 1 + i, D_a u0_i at
// 2 + 2 nd + i nd + a, L u0_i + G0_i/3 at 2 + 4 nd + nd^2 + i
__host__ __device__ constexpr int iso_fidx(int nd, int q) {
  return q < nd ? 1 + q : (q < nd + nd * nd ? 2 + 2 * nd + (q - nd) : 2 + 4 * nd + nd * nd + (q - nd - nd * nd));
}
template <typename R>
struct IsoBase {
  const R* bd;             // base data: field f at bd + f npts (general: [point], profile: [j nx])
  unsigned gmask, pmask;   // bit q: iso field q general / a y profile (neither: zero)
  R Tp, Ts;                // dT/dp, dT/ds
  R p0, ip0, T0, rho, irho, irT;   // irT = 1/(rho T0)
  R mu0, muT, lam0;        // mu(T0), mu'(T0), c_p mu(T0)/Pr
  R igam, icp;             // 1/gamma, 1/c_p
};
template <typename R>
hipError_t launch_jv_iso(const OpParams& p, const IsoBase<R>& ib, const R* x, R* y, int nrhs, R shift,
                         const int* active, hipStream_t s, long long sX, long long sY, const double* shifts,
                         long long sA, int nzc);
// flags[0] |= 1 if p0 or s0 differ anywhere from their value at point 0;
// for the iso_fields(ndim) base-data fields fidx[q]: flags[1] |= 1 << q if
// the field is non-zero somewhere, flags[2] |= 1 << q if it differs from
// its value at (x = 0, z = 0) of the same row somewhere
hipError_t launch_iso_classify(const OpParams& p, const double* base, const double* bdata, const int* fidx,
                               int nf, int* flags, hipStream_t s);

// Kernel launchers (all enqueue on the given stream; no synchronisation).
// base holds the nv base fields followed by three pointwise fields T0, dT/dp,
// dT/ds (all with walls); bdata the per-point base-state derivative data of
// launch_base_data (base_data_fields(ndim) fields).
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
// stage z4, stage z1, iso z32, iso z16, iso z4, iso z1 (zN: N planes per
// workgroup; shallow ones give small 3D grids enough workgroups; the iso
// kernels need a base state of uniform thermodynamic state)
constexpr int JV_NVARIANTS = 12;
constexpr bool jv_variant_is_iso(int v) { return v >= 8 && v < 12; }
template <typename R>
hipError_t launch_jv_pert(const OpParams& p, const R* base, const R* bdata, const R* x, R* y, int nrhs, R shift,
                          const int* active, hipStream_t s, long long sX = 0, long long sY = 0,
                          const double* shifts = nullptr, long long sA = 0, int variant = -1);
// A batch of systems in one launch: system r reads x + r*sX, writes y + r*sY
// with the shift shifts_dev[r] (device array; shifts_host holds the same
// values on the host).
template <typename R>
hipError_t launch_jv_batch(const OpParams& p, const R* base, const R* bdata, const R* x, R* y, int nsys,
                           long long sX, long long sY, const double* shifts_host, const double* shifts_dev,
                           const int* active, long long sA, hipStream_t s, int variant = -1);
hipError_t launch_base_data(const OpParams& p, const double* base, double* bdata, hipStream_t s);
// The compact-derivative operator (compact.hip): y = (J - shift I) x one
// system at a time through the workspace p.cwork, and its base data.
template <typename R>
hipError_t launch_jv_compact(const OpParams& p, const R* base, const R* bdata, const R* x, R* y, int nrhs, R shift,
                             const int* active, hipStream_t s, long long sX, long long sY, const double* shifts,
                             long long sA);
hipError_t launch_base_data_compact(const OpParams& p, const double* base, double* bdata, hipStream_t s);
size_t compact_work_elems(int ndim, long long npts);
size_t compact_table_elems(const OpParams& p);
void compact_tables(const OpParams& p, std::vector<double>& t64);
// Operator y = (J - shift I) x for nrhs vectors with the kernel variant given
// (-1: the precision's default).
template <typename R>
hipError_t launch_jv(const OpParams& p, const R* base, const R* bdata, const R* x, R* y, int nrhs, R shift,
                     const int* active, hipStream_t s, int variant = -1);

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

// Tangent-linear Navier-Stokes operator: y = (J(q0) - shift I) x.
//
// J is the exact derivative of the discrete right-hand side N(q) of the
// compressible Navier-Stokes equations in (p, u_i, s) form (Section
// "Governing equations", eq. navier_stokes), i.e. the operator N_lin that
// the Frechet quotient of eq. frechet approximates.  The discretisation:
//   * explicit central differences, 6th order in the interior, 4th and 2nd
//     order on the second and first rows next to a wall; mixed derivatives
//     are products of first differences;
//   * viscous terms in expanded form, d_j tau_ij = mu L u_i + mu/3 G_i +
//     mu'(T)[D_j T (D_j u_i + D_i u_j) - 2/3 D_i T D_k u_k] with
//     G_i = D2_i u_i + sum_{j!=i} D_i D_j u_j, heat flux lambda L T +
//     lambda'(T) |D T|^2, dissipation mu (2 s_ij s_ij - 2/3 s_kk^2);
//   * the pressure equation with the material derivative and the heat
//     terms (gamma-1)(Q+Phi); the entropy equation with +(Q+Phi)/(rho T);
//   * Sutherland viscosity, lambda = c_p mu/Pr, ideal gas.
// Linearisation: every product is differentiated by the product rule; the
// temperature perturbation T' = T_p p' + T_s s' is formed pointwise before
// it is differentiated; base-state derivatives are the discrete ones.

#include "jv_common.h"

namespace sa {
namespace {

__global__ void base_derive_kernel(OpParams op, double* __restrict__ base, float* __restrict__ base32,
                                   int* __restrict__ flag) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= op.npts) return;
  const int nv = op.ndim + 2;
  const double p = base[id];
  const double s = base[(long long)(nv - 1) * op.npts + id];
  bool bad = !(p > 0.0) || !isfinite(p);
  for (int f = 0; f < nv; ++f) bad = bad || !isfinite(base[(long long)f * op.npts + id]);
  // rho = (p/p_ref)^(1/gamma) exp(-s/c_p), T = p/(rho R)
  const double rho = exp(log(p / op.p_ref) / op.gamma - s / op.cp);
  const double T = p / (rho * op.R);
  const double Tp = T / p * (1.0 - 1.0 / op.gamma);
  const double Ts = T / op.cp;
  base[(long long)nv * op.npts + id] = T;
  base[(long long)(nv + 1) * op.npts + id] = Tp;
  base[(long long)(nv + 2) * op.npts + id] = Ts;
  for (int f = 0; f < nv + 3; ++f)
    base32[(long long)f * op.npts + id] = (float)base[(long long)f * op.npts + id];
  if (bad) atomicOr(flag, 1);
}

// Exact classification of the base state (see launch_iso_classify).
struct IsoIdx {
  int q[ISO_MAXF];
};
__global__ void iso_classify_kernel(OpParams op, const double* __restrict__ base, const double* __restrict__ bdata,
                                    IsoIdx fi, int nf, int* __restrict__ flags) {
  __shared__ int sf[3];
  if (threadIdx.x < 3) sf[threadIdx.x] = 0;
  __syncthreads();
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id < op.npts) {
    const int nv = op.ndim + 2;
    int nonuni = 0, nz = 0, var = 0;
    if (base[id] != base[0] || base[(long long)(nv - 1) * op.npts + id] != base[(long long)(nv - 1) * op.npts])
      nonuni = 1;
    const int j = (int)((id / op.nx) % op.ny);
    for (int q = 0; q < nf; ++q) {
      const double* f = bdata + (long long)fi.q[q] * op.npts;
      const double v = f[id];
      if (v != 0.0) nz |= 1 << q;
      if (v != f[(long long)j * op.nx]) var |= 1 << q;
    }
    if (nonuni) atomicOr(&sf[0], 1);
    if (nz) atomicOr(&sf[1], nz);
    if (var) atomicOr(&sf[2], var);
  }
  __syncthreads();
  if (threadIdx.x < 3 && sf[threadIdx.x]) atomicOr(&flags[threadIdx.x], sf[threadIdx.x]);
}

}  // namespace

hipError_t launch_iso_classify(const OpParams& p, const double* base, const double* bdata, const int* fidx, int nf,
                               int* flags, hipStream_t s) {
  if (nf > ISO_MAXF) return hipErrorInvalidValue;
  IsoIdx fi{};
  for (int q = 0; q < nf; ++q) fi.q[q] = fidx[q];
  const int threads = 256;
  const long long blocks = (p.npts + threads - 1) / threads;
  iso_classify_kernel<<<dim3((unsigned)blocks), dim3(threads), 0, s>>>(p, base, bdata, fi, nf, flags);
  return hipGetLastError();
}

hipError_t launch_base_derive(const OpParams& p, double* base, float* base32, int* flag,
                              hipStream_t s) {
  const int threads = 256;
  const long long blocks = (p.npts + threads - 1) / threads;
  base_derive_kernel<<<dim3((unsigned)blocks), dim3(threads), 0, s>>>(p, base, base32, flag);
  return hipGetLastError();
}

}  // namespace sa

namespace sa {

template <typename R>
hipError_t launch_jv_pert(const OpParams& p, const R* base, const R* bdata, const R* x, R* y, int nrhs, R shift,
                          const int* active, hipStream_t s, long long sX, long long sY, const double* shifts,
                          long long sA, int variant) {
  if (p.scheme == 1) return launch_jv_compact<R>(p, base, bdata, x, y, nrhs, shift, active, s, sX, sY, shifts, sA);
  if (variant < 0 || variant >= JV_NVARIANTS) variant = sizeof(R) == 8 ? 0 : 2;
  // kernel (0 prefetch, 1 stage) and z planes per workgroup of each variant
  // an iso variant on a base state outside that class: the default kernel
  const IsoBase<R>* ib = static_cast<const IsoBase<R>*>(p.iso[sizeof(R) == 8 ? 0 : 1]);
  if (jv_variant_is_iso(variant) && !ib) variant = sizeof(R) == 8 ? 0 : 2;
  static constexpr int kind[JV_NVARIANTS] = {0, 0, 1, 1, 0, 0, 1, 1, 2, 2, 2, 2};
  static constexpr int depth[JV_NVARIANTS] = {32, 16, 16, 32, 4, 1, 4, 1, 32, 16, 4, 1};
  const int nzc = depth[variant];
  if (kind[variant] == 2)
    return launch_jv_iso<R>(p, *ib, x, y, nrhs, shift, active, s, sX, sY, shifts, sA, nzc);
  if (kind[variant] == 0)
    return launch_jv_prefetch<R>(p, base, bdata, x, y, nrhs, shift, active, s, sX, sY, shifts, sA, nzc);
  return launch_jv_stage<R>(p, base, bdata, x, y, nrhs, shift, active, s, sX, sY, shifts, sA, nzc);
}

template <typename R>
hipError_t launch_jv(const OpParams& p, const R* base, const R* bdata, const R* x, R* y, int nrhs, R shift,
                     const int* active, hipStream_t s, int variant) {
  return launch_jv_pert<R>(p, base, bdata, x, y, nrhs, shift, active, s, 0, 0, nullptr, 0, variant);
}

template <typename R>
hipError_t launch_jv_batch(const OpParams& p, const R* base, const R* bdata, const R* x, R* y, int nsys,
                           long long sX, long long sY, const double* shifts_host, const double* shifts_dev,
                           const int* active, long long sA, hipStream_t s, int variant) {
  (void)shifts_host;
  return launch_jv_pert<R>(p, base, bdata, x, y, nsys, R(0), active, s, sX, sY, shifts_dev, sA, variant);
}

template hipError_t launch_jv_batch<double>(const OpParams&, const double*, const double*, const double*, double*,
                                            int, long long, long long, const double*, const double*, const int*,
                                            long long, hipStream_t, int);
template hipError_t launch_jv_batch<float>(const OpParams&, const float*, const float*, const float*, float*, int,
                                           long long, long long, const double*, const double*, const int*,
                                           long long, hipStream_t, int);

template hipError_t launch_jv<double>(const OpParams&, const double*, const double*, const double*, double*,
                                      int, double, const int*, hipStream_t, int);
template hipError_t launch_jv<float>(const OpParams&, const float*, const float*, const float*, float*, int,
                                     float, const int*, hipStream_t, int);

}  // namespace sa

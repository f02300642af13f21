// Base-state derivative data (sa_base_set): the per-point fields the
// operator kernels read instead of differentiating q0 in every product --
// p0, u0_i, T0, D p0, D u0, D s0, D T0, L u0 + G0/3, L T0 -- computed with
// the same discrete stencils as the operator (jv.hip).
//
// A workgroup owns a TX x TY column tile and marches over a chunk of z
// planes.  For each plane:
//   1. the plane with a 3-point xy halo is staged in LDS (base p, u_i, s, T);
//   2. z-derivatives come from the thread's own column (loads of planes
//      k +- 1..3), accumulated on the fly;
//   3. mixed derivatives are first differences of staged first-derivative
//      fields (the tensor-product differences commute):
//        G_x = D2_x u + D_x (D_y v + D_z w)
//        G_y = D2_y v + D_y (D_x u + D_z w)
//        G_z = D2_z w + D_x (D_z u) + D_y (D_z v)
//      so the staged fields need only an x halo (D_y v + D_z w, D_z u) or a
//      y halo (D_x u + D_z w, D_z v); their halo values are computed by
//      spare threads;
//   4. the fields are written to the base-data array.
#include "jv_common.h"

namespace sa {
namespace {

constexpr int TX = 32;
constexpr int TY = 8;
constexpr int PW = TX + 6;
constexpr int PH = TY + 6;
constexpr int NT = TX * TY;
constexpr int NZC = 8;       // z planes per workgroup

// Periodic index of a in [-n, 2n).  Indices beyond n + 3 only feed points
// outside the grid (tiles are padded), so they are clamped into range.
template <typename R>
__device__ __forceinline__ int wrap(int a, int n) {
  return a < 0 ? a + n : (a >= n ? min(a - n, n - 1) : a);
}


template <int ND>
constexpr int bdata_count() { return 1 + ND + 1 + ND + ND * ND + ND + ND + ND + 1; }

template <typename R, int ND>
__global__ void __launch_bounds__(NT) base_data_kernel(OpParams op, const R* __restrict__ base,
                                                       R* __restrict__ bdata) {
  constexpr int NF = ND + 3;
  constexpr int NSET = 1;
  constexpr int NPL = NSET * NF;                    // staged plane fields
  __shared__ R sP[NPL][PH][PW];
  // x-staged: [set][0: D_y v + D_z w, 1: D_z u][TY][PW]; y-staged: [set][0: D_x u + D_z w, 1: D_z v][PH][TX]
  __shared__ R sX[NSET][2][TY][PW];
  __shared__ R sY[NSET][2][PH][TX];
  auto is_pert = [](int) -> bool { return false; };   // only the base state is differentiated

  const int tid = threadIdx.x;
  const int ti = tid % TX, tj = tid / TX;
  const int i0 = blockIdx.x * TX, j0 = blockIdx.y * TY;
  const int i = i0 + ti, j = j0 + tj;
  const int nx = op.nx, ny = op.ny, nz = op.nz;
  const long long npts = op.npts;
  const bool inside = i < nx && j < ny;
  const R ihx = R(op.ihx), ihz = R(op.ihz);
  // y metric of the own row (uniform or stretched rows)
  const R* ymt = ymet<R>(op);
  const int jm = j < ny ? j : ny - 1;
  const R my1 = ymt[jm], my2 = ymt[ny + jm], my4 = ymt[2 * ny + jm];

  const Axis<R> ax = axis_coefs<R>(6);
  const Axis<R> ayc = axis_coefs<R>(wall_row_order(j < ny ? j : ny - 1, ny, op.bcy));
  const Axis<R> az = axis_coefs<R>(6);

  const int kbeg = ND == 3 ? blockIdx.z * NZC : 0;
  const int kend = ND == 3 ? min(nz, kbeg + NZC) : 1;

  // global row index of a staged row (clamped at walls, wrapped if periodic)
  auto grow = [&](int jj) -> int {
    int g = j0 - 3 + jj;
    if (op.bcy == 0) return wrap<R>(g, ny);
    return g < 0 ? 0 : (g > ny - 1 ? ny - 1 : g);
  };
  auto is_wall = [&](int g) -> bool { return op.bcy == 1 && (g == 0 || g == ny - 1); };

  // base field f (p, u_i, s, then T) at flat point p
  auto loadf = [&](bool, int f, long long p, bool) -> R { return base[(long long)f * npts + p]; };

  // D_z of field f of one set at column (ii, gj) plane k (global loads)
  auto dz1 = [&](bool pert, int f, int gi, int gj, int k, bool wall) -> R {
    R acc = R(0);
#pragma unroll
    for (int m = 1; m <= 3; ++m) {
      const long long pp = ((long long)wrap<R>(k + m, nz) * ny + gj) * nx + gi;
      const long long pm = ((long long)wrap<R>(k - m, nz) * ny + gj) * nx + gi;
      acc += az.c1[m - 1] * (loadf(pert, f, pp, wall) - loadf(pert, f, pm, wall));
    }
    return acc * ihz;
  };

  for (int k = kbeg; k < kend; ++k) {
    __syncthreads();
    // 1. stage the plane with its xy halo
    for (int t = tid; t < PW * PH; t += NT) {
      const int ii = t % PW, jj = t / PW;
      const int gi = wrap<R>(i0 - 3 + ii, nx);
      const int gj = grow(jj);
      const bool wall = is_wall(gj);
      const long long p = ((long long)k * ny + gj) * nx + gi;
#pragma unroll
      for (int s = 0; s < NSET; ++s)
#pragma unroll
        for (int f = 0; f < NF; ++f) sP[s * NF + f][jj][ii] = loadf(is_pert(s), f, p, is_pert(s) && wall);
    }
    // 2. z-derivatives of the own column (registers)
    R dz[NSET][NF], d2z[NSET][ND + 1];
    if (ND == 3) {
      const int gi = wrap<R>(i, nx), gj = grow(tj + 3);
      const bool wall = is_wall(gj);
#pragma unroll
      for (int s = 0; s < NSET; ++s) {
#pragma unroll
        for (int f = 0; f < NF; ++f) {
          R a1 = R(0), a2 = R(0);
#pragma unroll
          for (int m = 1; m <= 3; ++m) {
            const long long pp = ((long long)wrap<R>(k + m, nz) * ny + gj) * nx + gi;
            const long long pm = ((long long)wrap<R>(k - m, nz) * ny + gj) * nx + gi;
            const R vp = loadf(is_pert(s), f, pp, wall), vm = loadf(is_pert(s), f, pm, wall);
            a1 += az.c1[m - 1] * (vp - vm);
            a2 += az.c2[m - 1] * (vp + vm);
          }
          dz[s][f] = a1 * ihz;
          __builtin_amdgcn_sched_barrier(0);   // keep each field's loads together (register pressure)
          // second derivative for u_i (f = 1..ND) and T (f = ND+2): index f-1 / ND
          if (f >= 1 && f <= ND) d2z[s][f - 1] = a2;
          if (f == ND + 2) d2z[s][ND] = a2;
        }
      }
    }
    __syncthreads();
    // 3a. halo values of the staged first-derivative fields (spare work)
    if (ND == 3) {
      const int nxh = 6 * TY, nyh = 6 * TX;
      for (int t = tid; t < nxh + nyh; t += NT) {
        if (t < nxh) {
          // x-halo column: ii in {0,1,2, TX+3..TX+5}, row tj2
          const int c = t % 6, tj2 = t / 6;
          const int ii = c < 3 ? c : TX + c;
          const int gi = wrap<R>(i0 - 3 + ii, nx);
          const int gj = grow(tj2 + 3);
          const bool wall = is_wall(gj);
          const Axis<R> ay2 = axis_coefs<R>(wall_row_order(gj, ny, op.bcy));
#pragma unroll
          for (int s = 0; s < NSET; ++s) {
            const int F0 = s * NF;
            R dyv = R(0);
#pragma unroll
            for (int m = 1; m <= 3; ++m)
              dyv += ay2.c1[m - 1] * (sP[F0 + 2][tj2 + 3 + m][ii] - sP[F0 + 2][tj2 + 3 - m][ii]);
            dyv *= ymt[gj];
            const R dzw = dz1(is_pert(s), 3, gi, gj, k, wall);
            const R dzu = dz1(is_pert(s), 1, gi, gj, k, wall);
            sX[s][0][tj2][ii] = dyv + dzw;
            sX[s][1][tj2][ii] = dzu;
          }
        } else {
          const int t2 = t - nxh;
          const int ti2 = t2 % TX, r = t2 / TX;
          const int jj = r < 3 ? r : TY + r;
          const int gi = wrap<R>(i0 + ti2, nx);
          const int gj = grow(jj);
          const bool wall = is_wall(gj);
#pragma unroll
          for (int s = 0; s < NSET; ++s) {
            const int F0 = s * NF;
            R dxu = R(0);
#pragma unroll
            for (int m = 1; m <= 3; ++m)
              dxu += ax.c1[m - 1] * (sP[F0 + 1][jj][ti2 + 3 + m] - sP[F0 + 1][jj][ti2 + 3 - m]);
            dxu *= ihx;
            const R dzw = dz1(is_pert(s), 3, gi, gj, k, wall);
            const R dzv = dz1(is_pert(s), 2, gi, gj, k, wall);
            sY[s][0][jj][ti2] = dxu + dzw;
            sY[s][1][jj][ti2] = dzv;
          }
        }
      }
    } else {
      // 2D: x-staged D_y v, y-staged D_x u
      const int nxh = 6 * TY, nyh = 6 * TX;
      for (int t = tid; t < nxh + nyh; t += NT) {
        if (t < nxh) {
          const int c = t % 6, tj2 = t / 6;
          const int ii = c < 3 ? c : TX + c;
          const int gj = grow(tj2 + 3);
          const Axis<R> ay2 = axis_coefs<R>(wall_row_order(gj, ny, op.bcy));
#pragma unroll
          for (int s = 0; s < NSET; ++s) {
            const int F0 = s * NF;
            R dyv = R(0);
#pragma unroll
            for (int m = 1; m <= 3; ++m)
              dyv += ay2.c1[m - 1] * (sP[F0 + 2][tj2 + 3 + m][ii] - sP[F0 + 2][tj2 + 3 - m][ii]);
            sX[s][0][tj2][ii] = dyv * ymt[gj];
          }
        } else {
          const int t2 = t - nxh;
          const int ti2 = t2 % TX, r = t2 / TX;
          const int jj = r < 3 ? r : TY + r;
#pragma unroll
          for (int s = 0; s < NSET; ++s) {
            const int F0 = s * NF;
            R dxu = R(0);
#pragma unroll
            for (int m = 1; m <= 3; ++m)
              dxu += ax.c1[m - 1] * (sP[F0 + 1][jj][ti2 + 3 + m] - sP[F0 + 1][jj][ti2 + 3 - m]);
            sY[s][0][jj][ti2] = dxu * ihx;
          }
        }
      }
    }
    // 3b. in-plane derivatives of the own point from LDS
    Pt<R, ND> P[NSET];
    const int cx = ti + 3, cy = tj + 3;
#pragma unroll
    for (int s = 0; s < NSET; ++s) {
      const int F0 = s * NF;
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        const R c0 = sP[F0 + f][cy][cx];
        R a1x = R(0), a2x = R(0), a1y = R(0), a2y = R(0);
#pragma unroll
        for (int m = 1; m <= 3; ++m) {
          const R xp = sP[F0 + f][cy][cx + m], xm = sP[F0 + f][cy][cx - m];
          const R yp = sP[F0 + f][cy + m][cx], ym = sP[F0 + f][cy - m][cx];
          a1x += ax.c1[m - 1] * (xp - xm);
          a2x += ax.c2[m - 1] * (xp + xm);
          a1y += ayc.c1[m - 1] * (yp - ym);
          a2y += ayc.c2[m - 1] * (yp + ym);
        }
        P[s].q[f] = c0;
        P[s].D[f][0] = a1x * ihx;
        P[s].D[f][1] = a1y * my1;
        if (ND == 3) P[s].D[f][ND - 1] = dz[s][f];
        // second derivatives: velocity components and T
        if ((f >= 1 && f <= ND) || f == ND + 2) {
          const R d2x = (ax.c0 * c0 + a2x) * (ihx * ihx);
          const R d2y = (ayc.c0 * c0 + a2y) * my2 + P[s].D[f][1] * my4;
          R d2zz = R(0);
          if (ND == 3) d2zz = (az.c0 * c0 + d2z[s][f == ND + 2 ? ND : f - 1]) * (ihz * ihz);
          const R L = d2x + d2y + d2zz;
          if (f == ND + 2) {
            P[s].LT = L;
          } else {
            P[s].Lu[f - 1] = L;
            P[s].G[f - 1] = (f == 1) ? d2x : (f == 2 ? d2y : d2zz);   // D2_i u_i; mixed parts added below
          }
        }
      }
    }
    // own staged values
    if (ND == 3) {
#pragma unroll
      for (int s = 0; s < NSET; ++s) {
        sX[s][0][tj][cx] = P[s].D[2][1] + P[s].D[3][ND - 1];   // D_y v + D_z w
        sX[s][1][tj][cx] = P[s].D[1][ND - 1];                  // D_z u
        sY[s][0][cy][ti] = P[s].D[1][0] + P[s].D[3][ND - 1];   // D_x u + D_z w
        sY[s][1][cy][ti] = P[s].D[2][ND - 1];                  // D_z v
      }
    } else {
#pragma unroll
      for (int s = 0; s < NSET; ++s) {
        sX[s][0][tj][cx] = P[s].D[2][1];   // D_y v
        sY[s][0][cy][ti] = P[s].D[1][0];   // D_x u
      }
    }
    __syncthreads();
    // 4. mixed parts of G
#pragma unroll
    for (int s = 0; s < NSET; ++s) {
      R gx = R(0), gy = R(0), gz1 = R(0), gz2 = R(0);
#pragma unroll
      for (int m = 1; m <= 3; ++m) {
        gx += ax.c1[m - 1] * (sX[s][0][tj][cx + m] - sX[s][0][tj][cx - m]);
        gy += ayc.c1[m - 1] * (sY[s][0][cy + m][ti] - sY[s][0][cy - m][ti]);
        if (ND == 3) {
          gz1 += ax.c1[m - 1] * (sX[s][1][tj][cx + m] - sX[s][1][tj][cx - m]);
          gz2 += ayc.c1[m - 1] * (sY[s][1][cy + m][ti] - sY[s][1][cy - m][ti]);
        }
      }
      P[s].G[0] += gx * ihx;
      P[s].G[1] += gy * my1;
      if (ND == 3) P[s].G[2] += gz1 * ihx + gz2 * my1;
    }
    // 5. the base data of the point
    const long long id = ((long long)k * ny + j) * nx + i;
    if (inside) {
      const Pt<R, ND>& b = P[0];
      int q = 0;
      auto put = [&](R v) { bdata[(long long)(q++) * npts + id] = v; };
      put(b.q[0]);
#pragma unroll
      for (int a = 0; a < ND; ++a) put(b.q[1 + a]);
      put(b.q[ND + 2]);
#pragma unroll
      for (int a = 0; a < ND; ++a) put(b.D[0][a]);
#pragma unroll
      for (int c2 = 0; c2 < ND; ++c2)
#pragma unroll
        for (int a = 0; a < ND; ++a) put(b.D[1 + c2][a]);
#pragma unroll
      for (int a = 0; a < ND; ++a) put(b.D[ND + 1][a]);
#pragma unroll
      for (int a = 0; a < ND; ++a) put(b.D[ND + 2][a]);
#pragma unroll
      for (int a = 0; a < ND; ++a) put(b.Lu[a] + b.G[a] * R(1.0 / 3.0));
      put(b.LT);
    }
  }
}

}  // namespace

int base_data_fields(int ndim) { return ndim == 2 ? bdata_count<2>() : bdata_count<3>(); }

hipError_t launch_base_data(const OpParams& p, const double* base, double* bdata, hipStream_t s) {
  dim3 grid((p.nx + TX - 1) / TX, (p.ny + TY - 1) / TY, p.ndim == 3 ? (p.nz + NZC - 1) / NZC : 1);
  if (p.ndim == 2)
    base_data_kernel<double, 2><<<grid, NT, 0, s>>>(p, base, bdata);
  else
    base_data_kernel<double, 3><<<grid, NT, 0, s>>>(p, base, bdata);
  return hipGetLastError();
}

}  // namespace sa

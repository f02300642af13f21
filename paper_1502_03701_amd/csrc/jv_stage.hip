// Perturbation-only operator kernel y = (J(q0) - shift I) x (staging
// variant, the FP32 default), used once the base state's derivative data exist (sa_base_set computes them
// with the tiled kernel of jv_tiled.hip).  Same discrete operator and the
// same pointwise algebra (jv_common.h); organised for throughput:
//   * a workgroup owns a TX x TY column tile and marches over NZC planes;
//   * each thread keeps its own column's perturbation values of planes
//     k-3 .. k+3 in a register queue (one new plane loaded per step), which
//     gives the z-derivatives without re-reading planes;
//   * the centre plane with a 3-point xy halo is staged in LDS for the x and
//     y derivatives;
//   * mixed derivatives are first differences of staged first derivatives
//     (G_x = D2_x u + D_x(D_y v + D_z w), G_y = D2_y v + D_y(D_x u + D_z w),
//     G_z = D2_z w + D_x(D_z u) + D_y(D_z v)); the z-derivatives on the halo
//     columns are formed from direct loads by spare threads;
//   * loads are branch-free (wall rows are clamped and masked), indices are
//     32-bit within a field;
//   * workgroups are numbered so that tiles adjacent in x run on the same
//     XCD (and share its L2).
// In FP32 this kernel fits two waves per SIMD, which hides latency better
// than the explicit prefetching of jv_prefetch.hip; in FP64 it does not.
#include "jv_common.h"

namespace sa {
namespace {

constexpr int TX = 32;
constexpr int TY = 8;
constexpr int PW = TX + 6;
constexpr int PH = TY + 6;
constexpr int NT = TX * TY;

constexpr int NXCD = 8;

// Periodic index of a in [-n, 2n).  Indices beyond n + 3 only feed points
// outside the grid (tiles are padded), so they are clamped into range.
__device__ __forceinline__ int wrapi(int a, int n) { return a < 0 ? a + n : (a >= n ? min(a - n, n - 1) : a); }

// A batch of systems shares one launch: blockIdx.z = sys * zchunks + chunk;
// system sys reads x + sys*sV, writes y + sys*sV, uses shifts[sys] (or the
// scalar shift) and the flag active[sys*sA].
template <typename R, int ND, int NZC>
__global__ void __launch_bounds__(NT) jv_stage_kernel(OpParams op, const R* __restrict__ base,
                                                     const R* __restrict__ bdata, const R* __restrict__ x,
                                                     R* __restrict__ y, R shift, const int* __restrict__ active,
                                                     long long strideX, long long strideY,
                                                     const double* __restrict__ shifts, long long sA, int zchunks,
                                                     int gx, int gy, int ntot) {
  // XCD-aware numbering: hardware block L runs on XCD L % 8; each XCD gets a
  // contiguous range of logical tiles (x fastest).
  int lb;
  {
    const int L = blockIdx.x;
    const int per = ntot / NXCD, rem = ntot % NXCD;
    const int xcd = L % NXCD, idx = L / NXCD;
    lb = xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
  }
  const int bxi = lb % gx;
  const int byi = (lb / gx) % gy;
  const int bz = lb / (gx * gy);
  const int sys = bz / zchunks;
  const int zc = bz % zchunks;
  if (active && !active[sys * sA]) return;
  x += sys * strideX;
  y += sys * strideY;
  if (shifts) shift = R(shifts[sys]);
  constexpr int NF = ND + 3;   // p, u_i, s, T'
  __shared__ R sP[NF][PH][PW];
  __shared__ R sX[2][TY][PW];  // D_y v + D_z w, D_z u  (x halo)
  __shared__ R sY[2][PH][TX];  // D_x u + D_z w, D_z v  (y halo)

  const int tid = threadIdx.x;
  const int ti = tid % TX, tj = tid / TX;
  const int nx = op.nx, ny = op.ny, nz = op.nz;
  const int i0 = bxi * TX, j0 = byi * TY;
  const int i = i0 + ti, j = j0 + tj;
  const int plane = nx * ny;
  const long long npts = op.npts;
  const bool inside = i < nx && j < ny;
  const bool wallbc = op.bcy == 1;
  const R ihx = R(op.ihx), ihz = R(op.ihz);
  // y metric of the own row (uniform or stretched rows)
  const R* ymt = ymet<R>(op);
  const int jm = j < ny ? j : ny - 1;
  const R my1 = ymt[jm], my2 = ymt[ny + jm], my4 = ymt[2 * ny + jm];
  const Axis<R> ax = axis_coefs<R>(6);
  const Axis<R> ayc = axis_coefs<R>(wall_row_order(j < ny ? j : ny - 1, ny, op.bcy));
  const Axis<R> az = axis_coefs<R>(6);

  const R* xf[ND + 2];
#pragma unroll
  for (int f = 0; f < ND + 2; ++f) xf[f] = x + (long long)f * npts;
  const R* Tp = base + (long long)(ND + 3) * npts;
  const R* Ts = base + (long long)(ND + 4) * npts;

  auto grow = [&](int jj) -> int {   // global row of a staged row
    const int g = j0 - 3 + jj;
    if (!wallbc) return wrapi(g, ny);
    return g < 0 ? 0 : (g > ny - 1 ? ny - 1 : g);
  };
  // perturbation field f (T' for f = ND+2) at flat index p, zero on walls
  auto pv = [&](int f, int p, bool wall) -> R {
    R v;
    if (f < ND + 2) {
      v = xf[f][p];
    } else {
      v = Tp[p] * xf[0][p] + Ts[p] * xf[ND + 1][p];
    }
    return wall ? R(0) : v;
  };
  auto dzcol = [&](int f, int colp, int k, bool wall) -> R {   // D_z from direct loads
    R acc = R(0);
#pragma unroll
    for (int m = 1; m <= 3; ++m)
      acc += az.c1[m - 1] * (pv(f, wrapi(k + m, nz) * plane + colp, wall) - pv(f, wrapi(k - m, nz) * plane + colp, wall));
    return acc * ihz;
  };

  const int kbeg = ND == 3 ? zc * NZC : 0;
  const int kend = ND == 3 ? min(nz, kbeg + NZC) : 1;
  const int gi_own = wrapi(i, nx);
  const int gj_own = grow(tj + 3);
  const bool wall_own = wallbc && (gj_own == 0 || gj_own == ny - 1);
  const int col_own = gj_own * nx + gi_own;

  // register queue: zq[f][m] = field f at plane k - 3 + m (own column)
  R zq[NF][7];
  if (ND == 3) {
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      const int p = wrapi(kbeg - 3 + m, nz) * plane + col_own;
#pragma unroll
      for (int f = 0; f < NF; ++f) zq[f][m] = pv(f, p, wall_own);
    }
  }

  for (int k = kbeg; k < kend; ++k) {
    if (ND == 3) {
      const int p = wrapi(k + 3, nz) * plane + col_own;
#pragma unroll
      for (int f = 0; f < NF; ++f) zq[f][6] = pv(f, p, wall_own);
    }
    __syncthreads();
    // stage plane k with its xy halo
    for (int t = tid; t < PW * PH; t += NT) {
      const int ii = t % PW, jj = t / PW;
      const int gj = grow(jj);
      const bool wall = wallbc && (gj == 0 || gj == ny - 1);
      const int p = k * plane + gj * nx + wrapi(i0 - 3 + ii, nx);
#pragma unroll
      for (int f = 0; f < NF; ++f) sP[f][jj][ii] = pv(f, p, wall);
    }
    __syncthreads();
    // halo values of the staged first-derivative fields
    {
      constexpr int NXH = 6 * TY;
      constexpr int NYH = 6 * TX;
      for (int t = tid; t < NXH + NYH; t += NT) {
        if (t < NXH) {
          const int c = t % 6, r = t / 6;
          const int ii = c < 3 ? c : TX + c;
          const int gj = grow(r + 3);
          const bool wall = wallbc && (gj == 0 || gj == ny - 1);
          const Axis<R> ay2 = axis_coefs<R>(wall_row_order(gj, ny, op.bcy));
          R dyv = R(0);
#pragma unroll
          for (int m = 1; m <= 3; ++m) dyv += ay2.c1[m - 1] * (sP[2][r + 3 + m][ii] - sP[2][r + 3 - m][ii]);
          R dzw = R(0), dzu = R(0);
          if (ND == 3) {
            const int colp = gj * nx + wrapi(i0 - 3 + ii, nx);
            dzw = dzcol(3, colp, k, wall);
            dzu = dzcol(1, colp, k, wall);
          }
          sX[0][r][ii] = dyv * ymt[gj] + dzw;
          sX[1][r][ii] = dzu;
        } else {
          const int t2 = t - NXH;
          const int c = t2 % TX, r = t2 / TX;
          const int jj = r < 3 ? r : TY + r;
          R dxu = R(0);
#pragma unroll
          for (int m = 1; m <= 3; ++m) dxu += ax.c1[m - 1] * (sP[1][jj][c + 3 + m] - sP[1][jj][c + 3 - m]);
          R dzw = R(0), dzv = R(0);
          if (ND == 3) {
            const int gj = grow(jj);
            const bool wall = wallbc && (gj == 0 || gj == ny - 1);
            const int colp = gj * nx + wrapi(i0 + c, nx);
            dzw = dzcol(3, colp, k, wall);
            dzv = dzcol(2, colp, k, wall);
          }
          sY[0][jj][c] = dxu * ihx + dzw;
          sY[1][jj][c] = dzv;
        }
      }
    }
    // own point: derivatives from LDS (x, y) and from the queue (z)
    Pt<R, ND> P;
    const int cx = ti + 3, cy = tj + 3;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const R c0 = sP[f][cy][cx];
      R a1x = R(0), a2x = R(0), a1y = R(0), a2y = R(0), a1z = R(0), a2z = R(0);
#pragma unroll
      for (int m = 1; m <= 3; ++m) {
        const R xp = sP[f][cy][cx + m], xm = sP[f][cy][cx - m];
        const R yp = sP[f][cy + m][cx], ym = sP[f][cy - m][cx];
        a1x += ax.c1[m - 1] * (xp - xm);
        a2x += ax.c2[m - 1] * (xp + xm);
        a1y += ayc.c1[m - 1] * (yp - ym);
        a2y += ayc.c2[m - 1] * (yp + ym);
        if (ND == 3) {
          const R zp = zq[f][3 + m], zm = zq[f][3 - m];
          a1z += az.c1[m - 1] * (zp - zm);
          a2z += az.c2[m - 1] * (zp + zm);
        }
      }
      P.q[f] = c0;
      P.D[f][0] = a1x * ihx;
      P.D[f][1] = a1y * my1;
      if (ND == 3) P.D[f][2] = a1z * ihz;
      if ((f >= 1 && f <= ND) || f == ND + 2) {
        const R d2x = (ax.c0 * c0 + a2x) * (ihx * ihx);
        const R d2y = (ayc.c0 * c0 + a2y) * my2 + P.D[f][1] * my4;
        const R d2z = ND == 3 ? (az.c0 * c0 + a2z) * (ihz * ihz) : R(0);
        const R L = d2x + d2y + d2z;
        if (f == ND + 2) {
          P.LT = L;
        } else {
          P.Lu[f - 1] = L;
          P.G[f - 1] = f == 1 ? d2x : (f == 2 ? d2y : d2z);
        }
      }
    }
    sX[0][tj][cx] = P.D[2][1] + (ND == 3 ? P.D[3][ND - 1] : R(0));
    sY[0][cy][ti] = P.D[1][0] + (ND == 3 ? P.D[3][ND - 1] : R(0));
    if (ND == 3) {
      sX[1][tj][cx] = P.D[1][ND - 1];
      sY[1][cy][ti] = P.D[2][ND - 1];
    }
    __syncthreads();
    {
      R gx = R(0), gy = R(0), gz1 = R(0), gz2 = R(0);
#pragma unroll
      for (int m = 1; m <= 3; ++m) {
        gx += ax.c1[m - 1] * (sX[0][tj][cx + m] - sX[0][tj][cx - m]);
        gy += ayc.c1[m - 1] * (sY[0][cy + m][ti] - sY[0][cy - m][ti]);
        if (ND == 3) {
          gz1 += ax.c1[m - 1] * (sX[1][tj][cx + m] - sX[1][tj][cx - m]);
          gz2 += ayc.c1[m - 1] * (sY[1][cy + m][ti] - sY[1][cy - m][ti]);
        }
      }
      P.G[0] += gx * ihx;
      P.G[1] += gy * my1;
      if (ND == 3) P.G[2] += gz1 * ihx + gz2 * my1;
    }
    if (inside) {
      const int id = k * plane + j * nx + i;
      const bool wallrow = wallbc && (j == 0 || j == ny - 1);
      R out[ND + 2];
      {
        Pt<R, ND> b;
        const R* bd = bdata + id;
        int q = 0;
        auto get = [&]() -> R {
          const R v = __builtin_nontemporal_load(bd + (long long)q * npts);   // streamed once
          ++q;
          return v;
        };
        b.q[0] = get();
#pragma unroll
        for (int a = 0; a < ND; ++a) b.q[1 + a] = get();
        b.q[ND + 2] = get();
        b.q[ND + 1] = R(0);
#pragma unroll
        for (int a = 0; a < ND; ++a) b.D[0][a] = get();
#pragma unroll
        for (int c2 = 0; c2 < ND; ++c2)
#pragma unroll
          for (int a = 0; a < ND; ++a) b.D[1 + c2][a] = get();
#pragma unroll
        for (int a = 0; a < ND; ++a) b.D[ND + 1][a] = get();
#pragma unroll
        for (int a = 0; a < ND; ++a) b.D[ND + 2][a] = get();
#pragma unroll
        for (int a = 0; a < ND; ++a) {
          b.Lu[a] = get();
          b.G[a] = R(0);
        }
        b.LT = get();
        tangent_point<R, ND>(b, P, op, out);
      }
#pragma unroll
      for (int f = 0; f < ND + 2; ++f)   // written once, read by another kernel: nontemporal
        __builtin_nontemporal_store(zero_on(wallrow, out[f] - shift * P.q[f]), y + ((long long)f * npts + id));
    }
    if (ND == 3) {
#pragma unroll
      for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int m = 0; m < 6; ++m) zq[f][m] = zq[f][m + 1];
    }
  }
}

}  // namespace

template <typename R>
hipError_t launch_jv_stage(const OpParams& p, const R* base, const R* bdata, const R* x, R* y, int nrhs, R shift,
                          const int* active, hipStream_t s, long long sX, long long sY, const double* shifts,
                          long long sA, int nzc) {
  const long long ndof = (long long)(p.ndim + 2) * p.npts;
  // 32-bit indices within the base data (the widest per-point array)
  if ((long long)base_data_fields(p.ndim) * p.npts >= (1LL << 31)) return hipErrorInvalidValue;
  if (nzc != 1 && nzc != 4 && nzc != 16 && nzc != 32) return hipErrorInvalidValue;
  const int zchunks = p.ndim == 3 ? (p.nz + nzc - 1) / nzc : 1;
  if (sX == 0) sX = ndof;   // right-hand sides one after another
  if (sY == 0) sY = ndof;
  const int gx = (p.nx + TX - 1) / TX, gy = (p.ny + TY - 1) / TY;
  const long long ntot = (long long)gx * gy * zchunks * nrhs;
  if (ntot >= (1LL << 31)) return hipErrorInvalidValue;
  dim3 grid((unsigned)ntot);
#define SA_LAUNCH(ND_, NZ_)                                                                                      \
  jv_stage_kernel<R, ND_, NZ_><<<grid, NT, 0, s>>>(p, base, bdata, x, y, shift, active, sX, sY, shifts, sA, zchunks, gx, gy, \
                                       (int)ntot)
  if (p.ndim == 2)
    SA_LAUNCH(2, 16);   // one plane: the chunk depth is irrelevant
  else if (nzc == 1)
    SA_LAUNCH(3, 1);
  else if (nzc == 4)
    SA_LAUNCH(3, 4);
  else if (nzc == 16)
    SA_LAUNCH(3, 16);
  else
    SA_LAUNCH(3, 32);
#undef SA_LAUNCH
  return hipGetLastError();
}

template hipError_t launch_jv_stage<double>(const OpParams&, const double*, const double*, const double*, double*,
                                           int, double, const int*, hipStream_t, long long, long long,
                                           const double*, long long, int);
template hipError_t launch_jv_stage<float>(const OpParams&, const float*, const float*, const float*, float*, int,
                                          float, const int*, hipStream_t, long long, long long, const double*,
                                          long long, int);

}  // namespace sa

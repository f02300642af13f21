// Operator kernel y = (J(q0) - shift I) x for base states of uniform
// thermodynamic state: p0 and s0 (hence T0, rho0, mu0, lambda0, dT/dp,
// dT/ds) the same at every grid point, with an arbitrary velocity field u0.
// The tanh mixing layer of Section "Model problem" (u0 = tanh(y), uniform
// p0 and T0), with or without a spanwise velocity perturbation, is of this
// class; sa_base_set detects it exactly and the autotuner then also times
// these variants.
//
// Same discrete operator as the general kernels (jv.hip): with D p0 = D s0 =
// D T0 = 0 and L T0 = 0 every term of the tangent-linear that multiplies a
// base-state pressure, entropy or temperature gradient vanishes, so the
// per-point base data reduce to u0_i, D_a u0_i and L u0_i + G0_i/3 (ND + ND^2
// + ND fields), and T' = T_p p' + T_s s' has uniform coefficients.  Each of
// these fields is classified once, exactly, as identically zero, a profile
// in y (the same value along x and z) or general: a zero field is not
// loaded, a profile is read from the base data's (x = 0, z = 0) column
// (cached), and only general fields stream from HBM.  For the workload
// 256x128x128 with spanwise noise, 7 of the 15 fields are general (w0, its
// three derivatives and the three viscous fields); for 2D parallel flows
// none is.
//
// Organisation: TX x TY column tiles marching over NZC planes with a
// register z-queue of the own column, the centre plane with its xy halo
// staged in LDS, XCD-aware tile numbering.  The in-plane mixed derivatives
// D_x D_y v and D_y D_x u are first differences of staged first derivatives.
// The mixed derivatives with z are taken in the other order, as z
// derivatives of in-plane ones (the x, y and z stencils act on different
// indices, so they commute exactly): D_z of E = (D_x w, D_y w, D_x u + D_y v)
// of the own column.  E of plane k+3 is formed from that plane's u, v, w
// staged with their xy halo, and E of planes k-3 .. k+3 lives in an LDS ring
// of the own thread, so no halo column is ever read along z.
#include "jv_common.h"

namespace sa {
namespace {

constexpr int TX = 16;
constexpr int TY = 16;
constexpr int PW = TX + 6;
constexpr int PH = TY + 6;
constexpr int NT = TX * TY;
constexpr int NHALO = PW * PH - NT;   // staged halo positions of a plane
constexpr int NXH = 6 * TY;           // x-strip positions needing D_y v
constexpr int NYH = 6 * TX;           // y-strip positions needing D_x u
constexpr int NRING = 6;              // E of planes k-3 .. k+3 (E[k-3] is read before E[k+3] is written)
static_assert(NHALO <= NT && NXH + NYH <= NT, "one halo position per thread");
constexpr int NXCD = 8;

__device__ __forceinline__ int wrapc(int a, int n) { return a < 0 ? a + n : (a >= n ? min(a - n, n - 1) : a); }

// FP32 full tiles: four wavefronts per SIMD (128 VGPRs, a 20-byte spill)
// run 8-10 % faster than three (145 VGPRs, none)
template <typename R, int ND, int NZC, bool FULL>
__global__ void __launch_bounds__(NT, sizeof(R) == 4 && FULL ? 4 : 2) jv_iso_kernel(OpParams op, IsoBase<R> ib, const R* __restrict__ x,
                                                    R* __restrict__ y, R shift, const int* __restrict__ active,
                                                    long long strideX, long long strideY,
                                                    const double* __restrict__ shifts, long long sA, int zchunks,
                                                    int gx, int gy, int ntot) {
  int lb;
  {
    const int L = blockIdx.x;
    const int per = ntot / NXCD, rem = ntot % NXCD;
    const int xcd = L % NXCD, idx = L / NXCD;
    lb = xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
  }
  const int bx = lb % gx;
  const int by = (lb / gx) % gy;
  const int bz = lb / (gx * gy);
  const int sys = bz / zchunks;
  const int zc = bz % zchunks;
  if (active && !active[sys * sA]) return;
  x += sys * strideX;
  y += sys * strideY;
  if (shifts) shift = R(shifts[sys]);
  constexpr int NF = ND + 2;   // p, u_i, s (T' = T_p p' + T_s s' is formed from their derivatives)
  constexpr int NB = iso_fields(ND);
  constexpr int N3 = ND == 3 ? 1 : 0;
  __shared__ R sP[NF][PH][PW];
  __shared__ R sX[TY][PW];                         // D_y v (x halo)
  __shared__ R sY[PH][TX];                         // D_x u (y halo)
  __shared__ R sN[N3 ? 3 : 1][N3 ? PH : 1][PW];    // u, v, w of plane k+3
  __shared__ R sE[N3 ? NRING : 1][3][NT];          // ring of E (own thread's slots)

  const int tid = threadIdx.x;
  const int ti = tid % TX, tj = tid / TX;
  const int nx = op.nx, ny = op.ny, nz = op.nz;
  const int i0 = bx * TX, j0 = by * TY;
  const int i = i0 + ti, j = j0 + tj;
  const int plane = nx * ny;
  const int npts = (int)op.npts;
  const bool inside = FULL || (i < nx && j < ny);
  const bool wallbc = op.bcy == 1;
  const R ihx = R(op.ihx), ihy = R(op.ihy), ihz = R(op.ihz);
  const Axis<R> ax = axis_coefs<R>(6);
  const Axis<R> ayc = axis_coefs<R>(wall_row_order(j < ny ? j : ny - 1, ny, op.bcy));
  const Axis<R> az = axis_coefs<R>(6);

  auto grow = [&](int jj) -> int {   // global row of a staged row
    const int g = j0 - 3 + jj;
    if (!wallbc) return wrapc(g, ny);
    return g < 0 ? 0 : (g > ny - 1 ? ny - 1 : g);
  };
  auto is_wall = [&](int g) -> bool { return wallbc && (g == 0 || g == ny - 1); };
  // x fields at flat index p; the wall rows are zeroed only when the values
  // are staged (no arithmetic right after the loads, so the wave does not
  // wait for them early)
  auto load_raw = [&](int p, R v[NF]) {
#pragma unroll
    for (int f = 0; f < NF; ++f) v[f] = x[f * npts + p];
  };
  auto finish_raw = [&](bool wall, R v[NF]) {
    if (wall) {
#pragma unroll
      for (int f = 0; f < NF; ++f) v[f] = R(0);
    }
  };

  const int col_own = grow(tj + 3) * nx + wrapc(i, nx);
  const bool wall_own = is_wall(grow(tj + 3));
  const int jrow = j < ny ? j : ny - 1;   // row of the own point (profiles)
  const bool has_h = tid < NHALO;
  int hii = 0, hjj = 0;
  if (tid < 6 * PW) {
    const int r = tid / PW;
    hii = tid % PW;
    hjj = r < 3 ? r : PH - 6 + r;
  } else if (has_h) {
    const int t2 = tid - 6 * PW;
    const int c = t2 % 6;
    hjj = 3 + t2 / 6;
    hii = c < 3 ? c : TX + c;
  }
  const int col_h = grow(hjj) * nx + wrapc(i0 - 3 + hii, nx);
  const bool wall_h = is_wall(grow(hjj));
  const bool has_d = tid < NXH + NYH;
  const bool dxs = tid < NXH;
  int dr, dc;
  if (dxs) {
    const int c = tid % 6;
    dr = tid / 6;
    dc = c < 3 ? c : TX + c;
  } else {
    const int t2 = has_d ? tid - NXH : 0;
    const int r = t2 / TX;
    dc = t2 % TX;
    dr = r < 3 ? r : TY + r;
  }
  const int gj_d = dxs ? grow(dr + 3) : grow(dr);
  const Axis<R> ayd = axis_coefs<R>(wall_row_order(gj_d, ny, op.bcy));

  const int kbeg = ND == 3 ? zc * NZC : 0;
  const int kend = ND == 3 ? min(nz, kbeg + NZC) : 1;

  R zq[NF][6];
  if (ND == 3) {
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      R v[NF];
      load_raw(wrapc(kbeg - 3 + m, nz) * plane + col_own, v);
      finish_raw(wall_own, v);
#pragma unroll
      for (int f = 0; f < NF; ++f) zq[f][m] = v[f];
    }
  }

  R hv[NF], hn[3], qn[NF], bq[NB];
  // u, v, w at the own thread's halo position of plane k (wrapped in z)
  auto load_halo_uvw = [&](int k) {
    const int p = wrapc(k, nz) * plane + col_h;
#pragma unroll
    for (int c = 0; c < 3; ++c) hn[c] = x[(1 + c) * npts + p];
  };
  auto finish_halo_uvw = [&]() {
    if (wall_h) {
#pragma unroll
      for (int c = 0; c < 3; ++c) hn[c] = R(0);
    }
  };
  auto load_plane = [&](int k) {
    load_raw(k * plane + col_h, hv);
    if (ND == 3) load_halo_uvw(k + 3);
    load_raw((ND == 3 ? wrapc(k + 3, nz) * plane : 0) + col_own, qn);
  };
  const int cx = ti + 3, cy = tj + 3;
  // u, v, w of a plane into sN (own point from own[], halo from hn)
  auto stage_uvw = [&](const R own[3]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) sN[c][cy][cx] = own[c];
    if (has_h) {
#pragma unroll
      for (int c = 0; c < 3; ++c) sN[c][hjj][hii] = hn[c];
    }
  };
  // E = (D_x w, D_y w, D_x u + D_y v) at the own point of the plane in sN
  auto form_E = [&](R e[3]) {
    R wx = R(0), wy = R(0), ux = R(0), vy = R(0);
#pragma unroll
    for (int m = 1; m <= 3; ++m) {
      wx += ax.c1[m - 1] * (sN[2][cy][cx + m] - sN[2][cy][cx - m]);
      wy += ayc.c1[m - 1] * (sN[2][cy + m][cx] - sN[2][cy - m][cx]);
      ux += ax.c1[m - 1] * (sN[0][cy][cx + m] - sN[0][cy][cx - m]);
      vy += ayc.c1[m - 1] * (sN[1][cy + m][cx] - sN[1][cy - m][cx]);
    }
    e[0] = wx * ihx;
    e[1] = wy * ihy;
    e[2] = ux * ihx + vy * ihy;
  };
  if (ND == 3) {
    // E of planes kbeg-3 .. kbeg+2 into ring slots 0 .. 5
    for (int m = 0; m < 6; ++m) {
      load_halo_uvw(kbeg - 3 + m);
      finish_halo_uvw();
      R own[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) own[c] = zq[1 + c][m];
      __syncthreads();
      stage_uvw(own);
      __syncthreads();
      R e[3];
      form_E(e);
#pragma unroll
      for (int c = 0; c < 3; ++c) sE[m][c][tid] = e[c];
    }
  }
  // base data of the own point: zero fields are not loaded, profiles come
  // from the (x = 0, z = 0) column, general fields stream once.  FP64: both
  // loads carry the non-temporal hint (the compiler merges them into one
  // load, which keeps a hint only if both have it), so that the base stream
  // does not push the centre plane's halo lines, first read three planes
  // earlier, out of the L2 (125.8 instead of 146 B/pt read); FP32, whose
  // halo fits the L2 anyway, ran slower with it.
  auto ld_base = [](const R* ptr) -> R {
    if constexpr (sizeof(R) == 8) return __builtin_nontemporal_load(ptr);
    else return *ptr;
  };
  // The masks and the field stride pass through an empty asm each plane so
  // that the per-field offsets are recomputed there (a few scalar
  // instructions) instead of being hoisted into 2 NB live scalar registers.
  auto load_base = [&](int k) {
    unsigned gm = ib.gmask, pm = ib.pmask;
    int np = npts;
    asm volatile("" : "+s"(gm), "+s"(pm), "+s"(np));
    const int pg = k * plane + col_own;
    const int pp = jrow * nx;
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int off = iso_fidx(ND, q) * np;
      if (gm >> q & 1u)
        bq[q] = ld_base(ib.bd + (off + pg));
      else if (pm >> q & 1u)
        bq[q] = ld_base(ib.bd + (off + pp));
      else
        bq[q] = R(0);
    }
  };
  for (int k = kbeg; k < kend; ++k) {
    const int pown = k * plane + col_own;
    load_plane(k);
    load_base(k);
    finish_raw(wall_h, hv);
    if (ND == 3) finish_halo_uvw();
    finish_raw(wall_own, qn);
    __syncthreads();
#pragma unroll
    for (int f = 0; f < NF; ++f) sP[f][cy][cx] = ND == 3 ? zq[f][3] : qn[f];
    if (has_h) {
#pragma unroll
      for (int f = 0; f < NF; ++f) sP[f][hjj][hii] = hv[f];
    }
    if (ND == 3) stage_uvw(&qn[1]);
    __syncthreads();
    if (has_d) {
      if (dxs) {
        R dyv = R(0);
#pragma unroll
        for (int m = 1; m <= 3; ++m) dyv += ayd.c1[m - 1] * (sP[2][dr + 3 + m][dc] - sP[2][dr + 3 - m][dc]);
        sX[dr][dc] = dyv * ihy;
      } else {
        R dxu = R(0);
#pragma unroll
        for (int m = 1; m <= 3; ++m) dxu += ax.c1[m - 1] * (sP[1][dr][dc + 3 + m] - sP[1][dr][dc + 3 - m]);
        sY[dr][dc] = dxu * ihx;
      }
    }
    // ---- base data of the point, and the quantities derived from it ----
    R u0[ND], Du0[ND][ND], vis[ND];
#pragma unroll
    for (int a = 0; a < ND; ++a) u0[a] = bq[a];
#pragma unroll
    for (int c2 = 0; c2 < ND; ++c2)
#pragma unroll
      for (int a = 0; a < ND; ++a) Du0[c2][a] = bq[ND + c2 * ND + a];
#pragma unroll
    for (int a = 0; a < ND; ++a) vis[a] = bq[ND + ND * ND + a];
    R th0 = R(0), S00 = R(0);
#pragma unroll
    for (int a = 0; a < ND; ++a) th0 += Du0[a][a];
#pragma unroll
    for (int a = 0; a < ND; ++a)
#pragma unroll
      for (int b = 0; b < ND; ++b) {
        const R s0 = R(0.5) * (Du0[a][b] + Du0[b][a]);
        S00 += s0 * s0;
      }
    const R phiS = R(2) * S00 - R(2.0 / 3.0) * th0 * th0;
    const R H0 = ib.mu0 * phiS;   // no heat flux: T0 is uniform

    // ---- derivatives of the own point's fields: x, y from LDS, z from the
    // queue; the tangent-linear is accumulated as each field is done ----
    auto stencil = [&](int f, R& c0, R D[ND], R& L, R& d2own, int own) {
      c0 = sP[f][cy][cx];
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
          const R zp = m == 3 ? qn[f] : zq[f][3 + m], zm = zq[f][3 - m];
          a1z += az.c1[m - 1] * (zp - zm);
          a2z += az.c2[m - 1] * (zp + zm);
        }
      }
      D[0] = a1x * ihx;
      D[1] = a1y * ihy;
      if constexpr (ND == 3) D[2] = a1z * ihz;
      const R d2x = (ax.c0 * c0 + a2x) * (ihx * ihx);
      const R d2y = (ayc.c0 * c0 + a2y) * (ihy * ihy);
      const R d2z = ND == 3 ? (az.c0 * c0 + a2z) * (ihz * ihz) : R(0);
      L = d2x + d2y + d2z;
      d2own = own == 0 ? d2x : (own == 1 ? d2y : d2z);
    };
    const R gam = R(op.gamma);
    const R irho2 = ib.irho * ib.irho, irT2 = ib.irT * ib.irT;
    R acc0, accS, accU[ND], Hp;
    {
      // pressure and entropy, then the temperature perturbation
      // T' = T_p p' + T_s s' (uniform coefficients: its derivatives are
      // those combinations of the derivatives of p' and s')
      R pc, Dp[ND], Lp, sc, Ds[ND], Ls, dummy;
      stencil(0, pc, Dp, Lp, dummy, 0);
      stencil(ND + 1, sc, Ds, Ls, dummy, 0);
      R advp = R(0), advs = R(0);
#pragma unroll
      for (int a = 0; a < ND; ++a) {
        advp += u0[a] * Dp[a];
        advs += u0[a] * Ds[a];
      }
      const R Tpr = ib.Tp * pc + ib.Ts * sc;
      const R LTp = ib.Tp * Lp + ib.Ts * Ls;
      const R rhop = ib.rho * (pc * ib.ip0 * ib.igam - sc * ib.icp);   // rho_p p' + rho_s s'
      acc0 = -advp - gam * th0 * pc - shift * pc;
      Hp = ib.lam0 * LTp + ib.muT * Tpr * phiS;
      accS = -advs - H0 * (rhop * ib.T0 + ib.rho * Tpr) * irT2 - shift * sc;
#pragma unroll
      for (int i2 = 0; i2 < ND; ++i2) {
        R cp2 = R(0);
#pragma unroll
        for (int a = 0; a < ND; ++a) cp2 += (ib.Tp * Dp[a] + ib.Ts * Ds[a]) * (Du0[i2][a] + Du0[a][i2]);
        const R DTi = ib.Tp * Dp[i2] + ib.Ts * Ds[i2];
        const R Vt = ib.muT * Tpr * vis[i2] + ib.muT * (cp2 - R(2.0 / 3.0) * DTi * th0);
        accU[i2] = (Vt - Dp[i2]) * ib.irho - rhop * (ib.mu0 * vis[i2]) * irho2;
      }
    }
    // velocities: divergence, strain products, advection, viscous terms
    R thp = R(0), S0p = R(0);
    R dyv = R(0), dxu = R(0);
#pragma unroll
    for (int c = 0; c < ND; ++c) {
      R uc, Du[ND], Lu, d2c;
      stencil(1 + c, uc, Du, Lu, d2c, c);
      thp += Du[c];
      R advu = R(0);
#pragma unroll
      for (int a = 0; a < ND; ++a) {
        S0p += R(0.5) * (Du0[c][a] + Du0[a][c]) * Du[a];
        advu += u0[a] * Du[a];
      }
#pragma unroll
      for (int i2 = 0; i2 < ND; ++i2) accU[i2] -= uc * Du0[i2][c];
      accU[c] += -advu + ib.mu0 * ib.irho * (Lu + d2c * R(1.0 / 3.0)) - shift * uc;
      // first derivatives the in-plane mixed terms of G' need at the own point
      if (c == 0) dxu = Du[0];
      if (c == 1) dyv = Du[1];
    }
    Hp += ib.mu0 * (R(4) * S0p - R(4.0 / 3.0) * th0 * thp);
    acc0 += -gam * ib.p0 * thp;
    // D_z E at plane k; E[k+m] sits in ring slot (k - kbeg + 3 + m) mod 6
    R dzE[3] = {R(0), R(0), R(0)};
    if (ND == 3) {
      const int r0 = k - kbeg;
      const int sm3 = r0 % NRING, sp1 = (r0 + 4) % NRING, sm1 = (r0 + 2) % NRING;
      const int sp2 = (r0 + 5) % NRING, sm2 = (r0 + 1) % NRING;
      R e3[3];
      form_E(e3);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const R em3 = sE[sm3][c][tid];
        sE[sm3][c][tid] = e3[c];
        dzE[c] = (az.c1[0] * (sE[sp1][c][tid] - sE[sm1][c][tid]) + az.c1[1] * (sE[sp2][c][tid] - sE[sm2][c][tid]) +
                  az.c1[2] * (e3[c] - em3)) * ihz;
      }
    }
    sX[tj][cx] = dyv;
    sY[cy][ti] = dxu;
    __syncthreads();
    {
      // mixed parts of G'_i: D_x D_y v + D_z D_x w, D_y D_x u + D_z D_y w, D_z (D_x u + D_y v)
      R gxs = R(0), gys = R(0);
#pragma unroll
      for (int m = 1; m <= 3; ++m) {
        gxs += ax.c1[m - 1] * (sX[tj][cx + m] - sX[tj][cx - m]);
        gys += ayc.c1[m - 1] * (sY[cy + m][ti] - sY[cy - m][ti]);
      }
      const R cg = ib.mu0 * ib.irho * R(1.0 / 3.0);
      accU[0] += cg * (gxs * ihx + dzE[0]);
      accU[1] += cg * (gys * ihy + dzE[1]);
      if constexpr (ND == 3) accU[2] += cg * dzE[2];
    }
    if (ND == 3) {
#pragma unroll
      for (int f = 0; f < NF; ++f) {
#pragma unroll
        for (int m = 0; m < 5; ++m) zq[f][m] = zq[f][m + 1];
        zq[f][5] = qn[f];
      }
    }

    if (inside) {
      const bool wallrow = wallbc && (j == 0 || j == ny - 1);
      R out[ND + 2];
      out[0] = acc0 + (gam - R(1)) * Hp;
#pragma unroll
      for (int c = 0; c < ND; ++c) out[1 + c] = accU[c];
      out[ND + 1] = accS + Hp * ib.irT;
#pragma unroll
      for (int f = 0; f < ND + 2; ++f)
        __builtin_nontemporal_store(zero_on(wallrow, out[f]), y + (f * npts + pown));
    }
  }
}

}  // namespace

template <typename R>
hipError_t launch_jv_iso(const OpParams& p, const IsoBase<R>& ib, const R* x, R* y, int nrhs, R shift,
                         const int* active, hipStream_t s, long long sX, long long sY, const double* shifts,
                         long long sA, int nzc) {
  const long long ndof = (long long)(p.ndim + 2) * p.npts;
  if (ndof >= (1LL << 31)) return hipErrorInvalidValue;   // 32-bit indices within a vector
  if (nzc != 1 && nzc != 4 && nzc != 16 && nzc != 32) return hipErrorInvalidValue;
  const int zchunks = p.ndim == 3 ? (p.nz + nzc - 1) / nzc : 1;
  if (sX == 0) sX = ndof;
  if (sY == 0) sY = ndof;
  const int gx = (p.nx + TX - 1) / TX, gy = (p.ny + TY - 1) / TY;
  const long long ntot = (long long)gx * gy * zchunks * nrhs;
  if (ntot >= (1LL << 31)) return hipErrorInvalidValue;
  dim3 grid((unsigned)ntot);
#define SA_LAUNCH(ND_, NZ_, F_)                                                                              \
  jv_iso_kernel<R, ND_, NZ_, F_><<<grid, NT, 0, s>>>(p, ib, x, y, shift, active, sX, sY, shifts, sA, zchunks, \
                                                      gx, gy, (int)ntot)
  const bool full = p.nx % TX == 0 && p.ny % TY == 0;
  if (p.ndim == 2) {
    SA_LAUNCH(2, 16, false);
  } else if (nzc == 1) {
    if (full) SA_LAUNCH(3, 1, true); else SA_LAUNCH(3, 1, false);
  } else if (nzc == 4) {
    if (full) SA_LAUNCH(3, 4, true); else SA_LAUNCH(3, 4, false);
  } else if (nzc == 16) {
    if (full) SA_LAUNCH(3, 16, true); else SA_LAUNCH(3, 16, false);
  } else {
    if (full) SA_LAUNCH(3, 32, true); else SA_LAUNCH(3, 32, false);
  }
#undef SA_LAUNCH
  return hipGetLastError();
}

template hipError_t launch_jv_iso<double>(const OpParams&, const IsoBase<double>&, const double*, double*, int,
                                          double, const int*, hipStream_t, long long, long long, const double*,
                                          long long, int);
template hipError_t launch_jv_iso<float>(const OpParams&, const IsoBase<float>&, const float*, float*, int, float,
                                         const int*, hipStream_t, long long, long long, const double*, long long,
                                         int);

}  // namespace sa

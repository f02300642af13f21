// Block-Jacobi preconditioner (Section "Preconditioning"): local dense blocks
// of the operator assembled from operator calls, factored once, applied in
// every GMRES step.
//
//  * Extraction by coloured probing: blocks of one colour are more than the
//    stencil reach (3 cells) apart along some axis, so one product J e with
//    e = sum over those blocks of unit vector l gives column l of all of
//    them.  The products run through the operator kernel in the factor
//    precision, 16 probes per launch; each batch of probes resets its own
//    entries afterwards.
//  * Block b of shift s is B_b + diag_add I + noise_std E_b - s I with E_b
//    seeded standard normals (Philox4x32-10 + Box-Muller, one per entry),
//    kept in FP64, on the block's interior DOFs; its wall DOFs (not unknowns
//    of P J P: zero rows and columns in B_b) keep the identity, with no
//    noise or shift, so the inverse on the interior is that of the interior
//    part.  The factor kernel rounds once to the factor precision.
//  * One workgroup per (shift, block) factors a block in LDS by LU with
//    partial pivoting and stores L\U plus the row permutation: FP32 blocks
//    of order 16k by a blocked LU (one wavefront per block: 16-column panels
//    eliminated in registers, trailing updates on the matrix cores), other
//    blocks unblocked (wave-butterfly pivot search, three barriers per
//    elimination step).
//  * Factors are stored block-interleaved: 64 consecutive blocks form a
//    group whose entry t is contiguous over the blocks.  The apply solves
//    one block per lane, so each factor load is a coalesced row across the
//    wave; it gathers r_b from the struct-of-arrays vector, solves
//    L U z = P r and scatters z back; wall DOFs give 0.
#include <cmath>
#include <vector>

#include "sa_runtime.h"

namespace sa {
namespace {

struct BLayout {
  int nv, nx, ny, nz;
  int bx, by, bz;
  int nbx, nby, nbz;
  int cells, nb;
  long long nblocks, npts;
  int bcy;
};

// flat DOF index of local DOF l of block b; -1 for a wall DOF
__device__ __forceinline__ long long block_dof(const BLayout& L, long long b, int l, bool& wall) {
  const int ib = (int)(b % L.nbx);
  const int jb = (int)((b / L.nbx) % L.nby);
  const int kb = (int)(b / ((long long)L.nbx * L.nby));
  const int var = l / L.cells;
  const int cell = l % L.cells;
  const int cx = cell % L.bx;
  const int cy = (cell / L.bx) % L.by;
  const int cz = cell / (L.bx * L.by);
  const int i = ib * L.bx + cx, j = jb * L.by + cy, k = kb * L.bz + cz;
  wall = L.bcy == 1 && (j == 0 || j == L.ny - 1);
  return (((long long)var * L.nz + k) * L.ny + j) * L.nx + i;
}

// whether local DOF l of block b lies on a wall row (not an unknown of the
// operator P J P: its row and column of the block are zero, and the shifted
// block keeps the identity there)
__device__ __forceinline__ bool local_wall(const BLayout& L, long long b, int l) {
  const int jb = (int)((b / L.nbx) % L.nby);
  const int cy = ((l % L.cells) / L.bx) % L.by;
  const int j = jb * L.by + cy;
  return L.bcy == 1 && (j == 0 || j == L.ny - 1);
}

// The blocks of one probe colour: block (ib, jb, kb) has colour
// ((kb % cz) cy + (jb % cy)) cx + (ib % cx), so colour col holds the blocks
// with residues (rx, ry, rz) along the axes: mx x my x mz of them.
struct ColourSet {
  int rx, ry, rz, mx, my, mz;
  long long count;
};

ColourSet colour_set(const BLayout& L, int col, int cx, int cy, int cz) {
  ColourSet q;
  q.rx = col % cx;
  q.ry = (col / cx) % cy;
  q.rz = col / (cx * cy);
  q.mx = (L.nbx - q.rx + cx - 1) / cx;
  q.my = (L.nby - q.ry + cy - 1) / cy;
  q.mz = (L.nbz - q.rz + cz - 1) / cz;
  q.count = (long long)q.mx * q.my * q.mz;
  return q;
}

// block index of the idx-th block of the colour
__device__ __forceinline__ long long colour_block(const BLayout& L, const ColourSet& q, int cx, int cy, int cz,
                                                  long long idx) {
  const int ic = (int)(idx % q.mx);
  const int jc = (int)((idx / q.mx) % q.my);
  const int kc = (int)(idx / ((long long)q.mx * q.my));
  const int ib = q.rx + ic * cx, jb = q.ry + jc * cy, kb = q.rz + kc * cz;
  return ((long long)kb * L.nby + jb) * L.nbx + ib;
}

// e[r][dof(b, l0 + r)] = value for the blocks b of one colour, r < nprobe
template <typename F>
__global__ void probe_fill_kernel(BLayout L, ColourSet q, F* __restrict__ e, long long n, int cx, int cy, int cz,
                                  int l0, int nprobe, F value) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= q.count * nprobe) return;
  const long long b = colour_block(L, q, cx, cy, cz, t % q.count);
  const int r = (int)(t / q.count);
  bool wall;
  const long long d = block_dof(L, b, l0 + r, wall);
  e[(long long)r * n + d] = value;
}

// B[b][l0 + r][row] = y[r][dof(b, row)] for the blocks of one colour
// (column-major blocks)
template <typename F>
__global__ void probe_extract_kernel(BLayout L, ColourSet q, const F* __restrict__ y, long long n,
                                     double* __restrict__ B, int cx, int cy, int cz, int l0, int nprobe) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long per = (long long)L.nb * nprobe;
  if (t >= q.count * per) return;
  const long long b = colour_block(L, q, cx, cy, cz, t / per);
  const int rem = (int)(t % per);
  const int r = rem / L.nb;
  const int row = rem % L.nb;
  bool wall;
  const long long d = block_dof(L, b, row, wall);
  B[(b * L.nb + (l0 + r)) * L.nb + row] = (double)y[(long long)r * n + d];
}

// --- Philox4x32-10 (Salmon et al. 2011) ---
__device__ __forceinline__ void philox(unsigned c[4], unsigned k0, unsigned k1) {
  const unsigned M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    const unsigned long long p0 = (unsigned long long)M0 * c[0];
    const unsigned long long p1 = (unsigned long long)M1 * c[2];
    const unsigned hi0 = (unsigned)(p0 >> 32), lo0 = (unsigned)p0;
    const unsigned hi1 = (unsigned)(p1 >> 32), lo1 = (unsigned)p1;
    const unsigned n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

__device__ __forceinline__ double noise_entry(unsigned long long seed, long long b, int idx) {
  unsigned c[4] = {(unsigned)idx, (unsigned)((unsigned long long)b & 0xffffffffu),
                   (unsigned)((unsigned long long)b >> 32), 0u};
  philox(c, (unsigned)(seed & 0xffffffffu), (unsigned)(seed >> 32));
  const unsigned long long a = ((unsigned long long)c[0] | ((unsigned long long)c[1] << 32)) >> 11;
  const unsigned long long bb = ((unsigned long long)c[2] | ((unsigned long long)c[3] << 32)) >> 11;
  const double u1 = ((double)a + 1.0) * 0x1.0p-53;
  const double u2 = (double)bb * 0x1.0p-53;
  return sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}

// B[b] += noise_std * E_b   (E_b[r][c] at column-major position c*nb + r)
// on the rows and columns of interior DOFs
__global__ void add_noise_kernel(BLayout L, double* __restrict__ B, double noise_std, unsigned long long seed) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long per = (long long)L.nb * L.nb;
  if (t >= L.nblocks * per) return;
  const long long b = t / per;
  const int e = (int)(t % per);
  const int col = e / L.nb, row = e % L.nb;
  if (local_wall(L, b, row) || local_wall(L, b, col)) return;
  B[t] += noise_std * noise_entry(seed, b, row * L.nb + col);
}

// (block, shift) of a factorisation workgroup.  Hardware workgroup L runs on
// XCD L % 8; consecutive blocks are given to one XCD so that the 64 blocks of
// an interleaved output group merge their partial cache-line writes in that
// XCD's L2.
__device__ __forceinline__ void lu_work_item(long long nblocks, long long& b, int& s) {
  const long long ntot = (long long)gridDim.x;
  const long long L = blockIdx.x;
  const long long per = ntot / 8, rem = ntot % 8;
  const long long xcd = L % 8, idx = L / 8;
  const long long lb = xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
  b = lb % nblocks;
  s = (int)(lb / nblocks);
}

// Factor B_b + (diag_add - shift_s) I, one workgroup of 256 threads per
// (block, shift).  The block sits in LDS (column-major, nb x nb).  Per
// elimination step the first wave finds the pivot (first largest |a_ik|,
// i >= k) by a butterfly over its lanes, then all threads swap rows k and p,
// scale the column and update the trailing matrix (one element per thread
// and pass): three workgroup barriers per step.
template <typename F>
__global__ void __launch_bounds__(256) lu_kernel(BLayout L, const double* __restrict__ B, const double* __restrict__ shifts,
                                                 double diag_add, F* __restrict__ LU, int* __restrict__ perm,
                                                 int* __restrict__ singular) {
  extern __shared__ unsigned char smem[];
  F* A = reinterpret_cast<F*>(smem);            // nb x nb column-major
  __shared__ int s_perm[128];
  __shared__ int s_piv;
  const int nb = L.nb;
  const int tid = threadIdx.x;
  long long b;
  int s;
  lu_work_item(L.nblocks, b, s);
  const double dshift = diag_add - shifts[s];
  const double* Bb = B + b * nb * nb;
  // all of a thread's loads in flight together (at most 64 per thread)
  for (int t0 = 0; t0 < nb * nb; t0 += 256 * 16) {
    double v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int t = t0 + tid + 256 * q;
      v[q] = t < nb * nb ? Bb[t] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int t = t0 + tid + 256 * q;
      if (t < nb * nb) {
        const bool diag = t / nb == t % nb;
        A[t] = (F)(diag ? (local_wall(L, b, t % nb) ? 1.0 : v[q] + dshift) : v[q]);
      }
    }
  }
  for (int t = tid; t < nb; t += blockDim.x) s_perm[t] = t;
  __syncthreads();
  bool sing = false;
  for (int k = 0; k < nb; ++k) {
    if (tid < 64) {
      F best = F(-1);
      int bi = nb;
      for (int i = k + tid; i < nb; i += 64) {
        const F v = fabs(A[k * nb + i]);
        if (v > best) {
          best = v;
          bi = i;
        }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const F ov = __shfl_xor(best, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        if (ov > best || (ov == best && oi < bi)) {
          best = ov;
          bi = oi;
        }
      }
      if (tid == 0) {
        s_piv = bi < nb ? bi : k;
        if (!(best > F(0))) sing = true;
      }
    }
    __syncthreads();
    const int p = s_piv;
    if (p != k) {
      for (int c = tid; c < nb; c += blockDim.x) {
        const F t1 = A[c * nb + k];
        A[c * nb + k] = A[c * nb + p];
        A[c * nb + p] = t1;
      }
      if (tid == 0) {
        const int t2 = s_perm[k];
        s_perm[k] = s_perm[p];
        s_perm[p] = t2;
      }
    }
    __syncthreads();
    const F piv = A[k * nb + k];
    const F ipiv = piv != F(0) ? F(1) / piv : F(0);
    // trailing update with the scaled column: a_ic -= (a_ik / a_kk) a_kc
    const int rem = nb - k - 1;
    for (int t = tid; t < rem * rem; t += blockDim.x) {
      const int c = k + 1 + t / rem, i = k + 1 + t % rem;
      A[c * nb + i] -= A[k * nb + i] * ipiv * A[c * nb + k];
    }
    __syncthreads();
    for (int i = k + 1 + tid; i < nb; i += blockDim.x) A[k * nb + i] *= ipiv;
  }
  __syncthreads();
  if (sing) atomicOr(singular, 1);
  // block-interleaved output: group g = b / 64 holds entry t of its 64 blocks
  // contiguously, so that the apply (one lane per block) reads coalesced rows
  const long long g = b / 64;
  const int gl = (int)(b % 64);
  const long long ngroups = (L.nblocks + 63) / 64;
  F* out = LU + ((long long)s * ngroups + g) * nb * nb * 64 + gl;
  for (int t = tid; t < nb * nb; t += blockDim.x) out[(long long)t * 64] = A[t];
  int* pout = perm + ((long long)s * ngroups + g) * nb * 64 + gl;
  for (int t = tid; t < nb; t += blockDim.x) pout[t * 64] = s_perm[t];
}

// FP32 factors of orders that are multiples of 16 (the C3 blocks are 80):
// blocked right-looking LU, one wavefront per (block, shift), the block in
// LDS (column stride nb + 1).  Per 16-column panel: unblocked elimination of
// the panel in registers with partial pivoting (wave butterfly for the
// pivot, the row exchanges then applied to the other columns), the
// triangular solve U12 = L11^-1 A12 (a lane per column), and the
// trailing update A22 -= L21 U12 on the matrix cores: 16 x 16 output tiles,
// four v_mfma_f32_16x16x4f32 each (K = 16).  Operand layout of that
// instruction for lane l: A[i][k] with i = l % 16, k = l / 16; B[k][j] with
// j = l % 16, k = l / 16; accumulator v of D[i][j] with i = 4 (l / 16) + v,
// j = l % 16.
typedef float floatx4 __attribute__((ext_vector_type(4)));
// Two wavefronts per factorisation: the first eliminates each panel, both
// share the row exchanges, the triangular solve, the trailing update's tiles
// and the block's load and store.
constexpr int LU_MFMA_THREADS = 128;

// maximum of v over the wavefront (uniform result): prefix maxima within
// each row of 16 lanes by DPP row shifts (lanes without a source take
// INT_MIN), then the four row maxima from lanes 15, 31, 47, 63
__device__ __forceinline__ int wave_max_bits(int v) {
  v = max(v, __builtin_amdgcn_update_dpp((int)0x80000000, v, 0x111, 0xf, 0xf, false));   // row_shr:1
  v = max(v, __builtin_amdgcn_update_dpp((int)0x80000000, v, 0x112, 0xf, 0xf, false));   // row_shr:2
  v = max(v, __builtin_amdgcn_update_dpp((int)0x80000000, v, 0x114, 0xf, 0xf, false));   // row_shr:4
  v = max(v, __builtin_amdgcn_update_dpp((int)0x80000000, v, 0x118, 0xf, 0xf, false));   // row_shr:8
  const int r0 = __builtin_amdgcn_readlane(v, 15), r1 = __builtin_amdgcn_readlane(v, 31);
  const int r2 = __builtin_amdgcn_readlane(v, 47), r3 = __builtin_amdgcn_readlane(v, 63);
  return max(max(r0, r1), max(r2, r3));
}

__global__ void __launch_bounds__(LU_MFMA_THREADS) lu_mfma_kernel(BLayout L, const double* __restrict__ B,
                                                     const double* __restrict__ shifts, double diag_add,
                                                     float* __restrict__ LU, int* __restrict__ perm,
                                                     int* __restrict__ singular) {
  extern __shared__ unsigned char smem[];
  const int nb = L.nb;
  const int ld = nb + 1;   // odd column stride: lane-per-column accesses hit distinct banks
  float* A = reinterpret_cast<float*>(smem);   // nb x nb column-major, leading dimension ld
  __shared__ int s_perm[128];
  __shared__ int s_piv[16];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int NW = LU_MFMA_THREADS / 64;
  long long b;
  int s;
  lu_work_item(L.nblocks, b, s);
  const double dshift = diag_add - shifts[s];
  const double* Bb = B + b * nb * nb;
  // by columns (lane: rows lane and lane + 64), 10 columns = 20 loads in
  // flight per lane per batch (the block is 51 KB of FP64), the batches
  // shared out over the wavefronts; no index division
  const bool r1 = lane < nb, r2 = lane + 64 < nb;
  const int l1 = r1 ? lane : nb - 1;   // clamped rows: loads stay inside the block
  for (int c0l = 10 * wave; c0l < nb; c0l += 10 * NW) {
    double v[10][2];
#pragma unroll
    for (int q = 0; q < 10; ++q) {
      const int col = min(c0l + q, nb - 1);
      v[q][0] = Bb[(long long)col * nb + l1];
      v[q][1] = Bb[(long long)col * nb + (r2 ? lane + 64 : l1)];
    }
#pragma unroll
    for (int q = 0; q < 10; ++q) {
      const int col = c0l + q;
      if (col < nb && r1) {
        const double d0 = lane == col ? (local_wall(L, b, col) ? 1.0 : v[q][0] + dshift) : v[q][0];
        A[col * ld + lane] = (float)d0;
        if (r2) {
          const int row = lane + 64;
          const double d1 = row == col ? (local_wall(L, b, col) ? 1.0 : v[q][1] + dshift) : v[q][1];
          A[col * ld + row] = (float)d1;
        }
      }
    }
  }
  for (int t = tid; t < nb; t += LU_MFMA_THREADS) s_perm[t] = t;
  __syncthreads();
  bool sing = false;
  const int li = lane % 16, lk = lane / 16;
  for (int c0 = 0; c0 < nb; c0 += 16) {
    if (wave == 0) {
    // Panel elimination, columns c0 .. c0+15, in registers: lane l holds the
    // physical rows c0 + l (slot a) and c0 + 64 + l (slot b) of the panel.
    // Pivoting is implicit: rows are not exchanged inside the panel; each
    // row carries its current position (the row exchanges of partial
    // pivoting applied to positions), a chosen pivot row leaves the
    // candidates, and the rows are stored at their final positions after
    // the panel.  The exchanges (piv, in positions) are then applied to the
    // other columns as usual.
    float P[2][16];
    const int ra = c0 + lane, rb = c0 + 64 + lane;
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      P[0][c] = ra < nb ? A[(c0 + c) * ld + ra] : 0.0f;
      P[1][c] = rb < nb ? A[(c0 + c) * ld + rb] : 0.0f;
    }
    int posa = ra, posb = rb;                  // current positions of the lane's rows
    bool da = ra >= nb, db = rb >= nb;         // chosen as a pivot already (or no row)
    int piv[16];
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      const int k = c0 + kk;
      // pivot: the largest |a_ik| over the remaining rows, the one at the
      // smallest position on ties (a wave max of the magnitudes' bit
      // patterns, -1 marking no candidate)
      const float va = da ? -1.0f : fabsf(P[0][kk]);
      const float vb = db ? -1.0f : fabsf(P[1][kk]);
      const int wbits = wave_max_bits(__float_as_int(va > vb ? va : vb));
      const float wmax = __int_as_float(wbits);
      if (!(wmax > 0.0f)) sing = true;
      // the candidates holding the maximum; the smallest position wins
      const int ca = __float_as_int(va) == wbits ? posa : 0x7fffffff;
      const int cb = __float_as_int(vb) == wbits ? posb : 0x7fffffff;
      const int p = -wave_max_bits(-(ca < cb ? ca : cb));   // position of the pivot row
      // its lane and slot
      const unsigned long long ma = __ballot(!da && posa == p);
      const bool sp = ma == 0ull;
      const unsigned long long mp = sp ? __ballot(!db && posb == p) : ma;
      const int lp = __ffsll((long long)mp) - 1;
      piv[kk] = p;
      float urow[16];
#pragma unroll
      for (int c = kk; c < 16; ++c)
        urow[c] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(sp ? P[1][c] : P[0][c]), lp));
      // positions: the row at position k moves to p, the pivot row to k
      if (p != k) {
        if (posa == k) posa = p;
        if (posb == k) posb = p;
        if (lane == lp) {
          if (sp) posb = k;
          else posa = k;
        }
        if (lane == 0) {
          const int t2 = s_perm[k];
          s_perm[k] = s_perm[p];
          s_perm[p] = t2;
        }
      }
      if (lane == lp) {
        if (sp) db = true;
        else da = true;
      }
      const float ipiv = urow[kk] != 0.0f ? 1.0f / urow[kk] : 0.0f;
      if (!da) {
        const float l = P[0][kk] * ipiv;
        P[0][kk] = l;
#pragma unroll
        for (int c = kk + 1; c < 16; ++c) P[0][c] -= l * urow[c];
      }
      if (!db) {
        const float l = P[1][kk] * ipiv;
        P[1][kk] = l;
#pragma unroll
        for (int c = kk + 1; c < 16; ++c) P[1][c] -= l * urow[c];
      }
    }
    // the panel's rows at their final positions (a row position is unique)
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      if (ra < nb) A[(c0 + c) * ld + posa] = P[0][c];
      if (rb < nb) A[(c0 + c) * ld + posb] = P[1][c];
    }
    if (lane == 0) {
#pragma unroll
      for (int kk = 0; kk < 16; ++kk) s_piv[kk] = piv[kk];
    }
    }   // wave 0
    __syncthreads();
    // the panel's row exchanges on the other columns (a thread per column)
    for (int c = tid; c < nb - 16; c += LU_MFMA_THREADS) {
      const int col = c < c0 ? c : c + 16;
      float* Ac = A + col * ld;
#pragma unroll
      for (int kk = 0; kk < 16; ++kk) {
        const int k = c0 + kk, p = s_piv[kk];
        if (p != k) {
          const float t1 = Ac[k];
          Ac[k] = Ac[p];
          Ac[p] = t1;
        }
      }
    }
    __syncthreads();
    const int c1 = c0 + 16;
    if (c1 >= nb) break;
    // U12 = L11^-1 A12 (unit lower L11), a thread per column
    for (int c = c1 + tid; c < nb; c += LU_MFMA_THREADS) {
      float x[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) x[i] = A[c * ld + c0 + i];
#pragma unroll
      for (int j = 0; j < 16; ++j) {
#pragma unroll
        for (int i = j + 1; i < 16; ++i) x[i] -= A[(c0 + j) * ld + c0 + i] * x[j];
      }
#pragma unroll
      for (int i = 1; i < 16; ++i) A[c * ld + c0 + i] = x[i];
    }
    __syncthreads();
    // A22 -= L21 U12, 16 x 16 tiles on the matrix cores
    const int nt = (nb - c1) / 16;
    for (int t = wave; t < nt * nt; t += NW) {
      const int r0 = c1 + 16 * (t % nt), q0 = c1 + 16 * (t / nt);
      floatx4 acc;
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[v] = A[(q0 + li) * ld + r0 + 4 * lk + v];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const float a = -A[(c0 + 4 * kk + lk) * ld + r0 + li];    // -L21[r0+li][c0+4kk+lk]
        const float bv = A[(q0 + li) * ld + c0 + 4 * kk + lk];    // U12[c0+4kk+lk][q0+li]
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bv, acc, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) A[(q0 + li) * ld + r0 + 4 * lk + v] = acc[v];
    }
    __syncthreads();
  }
  if (sing && tid == 0) atomicOr(singular, 1);
  const long long g = b / 64;
  const int gl = (int)(b % 64);
  const long long ngroups = (L.nblocks + 63) / 64;
  float* out = LU + ((long long)s * ngroups + g) * nb * nb * 64 + gl;
  for (int col = wave; col < nb; col += NW) {
    if (r1) out[((long long)col * nb + lane) * 64] = A[col * ld + lane];
    if (r2) out[((long long)col * nb + lane + 64) * 64] = A[col * ld + lane + 64];
  }
  int* pout = perm + ((long long)s * ngroups + g) * nb * 64 + gl;
  for (int t = tid; t < nb; t += LU_MFMA_THREADS) pout[t * 64] = s_perm[t];
}

// z_b = U^{-1} L^{-1} (P r_b), one lane per block: a wavefront solves the 64
// blocks of one interleaved group, so every factor load is one coalesced
// 256-byte row across the wave, and the loads (independent of the solve)
// stream while the substitutions run.  The right-hand side / solution of a
// lane lives in LDS (column lane, conflict-free), solved in place.
// Dot-product form:
//   forward  y_i = (P r)_i - sum_{j<i} L_ij y_j      (unit lower)
//   backward z_i = (y_i - sum_{j>i} U_ij z_j) / U_ii
template <typename F, typename R>
__global__ void __launch_bounds__(64) apply_kernel(BLayout L, const F* __restrict__ LU, const int* __restrict__ perm,
                                                   int shift0, int shift_step, const R* __restrict__ r,
                                                   R* __restrict__ z, long long sV, const int* __restrict__ active,
                                                   long long sA) {
  const int rhs = blockIdx.y;
  if (active && !active[rhs * sA]) return;
  extern __shared__ unsigned char smem[];
  F* xs = reinterpret_cast<F*>(smem);   // [nb][64]: column lane is this lane's vector
  const int nb = L.nb;
  const int lane = threadIdx.x;
  const long long g = blockIdx.x;
  const long long b = g * 64 + lane;
  const bool valid = b < L.nblocks;
  const long long bb = valid ? b : L.nblocks - 1;   // padding lanes solve a real block, store nothing
  const long long ngroups = (L.nblocks + 63) / 64;
  const int shift = shift0 + rhs * shift_step;
  const R* rr = r + (long long)rhs * sV;
  R* zz = z + (long long)rhs * sV;
  const F* A = LU + ((long long)shift * ngroups + g) * nb * nb * 64 + lane;   // entry (i, j) at (j nb + i) 64
  const int* pg = perm + ((long long)shift * ngroups + g) * nb * 64 + lane;
  if (!valid) A = LU + ((long long)shift * ngroups + g) * nb * nb * 64 + (bb % 64);
  if (!valid) pg = perm + ((long long)shift * ngroups + g) * nb * 64 + (bb % 64);
  // gather the permuted right-hand side (P r_b)_i = r_b[p(i)] into LDS
  F* ys = xs;
  for (int i = 0; i < nb; ++i) {
    bool wall;
    const long long d = block_dof(L, bb, pg[(long long)i * 64], wall);
    ys[i * 64 + lane] = wall ? F(0) : (F)rr[d];
  }
  // Both substitutions go in chunks of RB rows: the updates from the rows
  // already solved are RB independent, contiguous loads per column (memory-
  // level parallelism for the one-pass stream of factors), then the RB x RB
  // diagonal block is solved in registers.  Rows past the end of a short last
  // chunk read clamped (valid) entries and are never stored, so every load is
  // unconditional and the compiler can issue them together.
  constexpr int RB = 16;
  auto entry = [&](int row, int col) -> F {   // factor entry, indices clamped into the block
    row = row < nb ? row : nb - 1;
    col = col < nb ? col : nb - 1;
    return __builtin_nontemporal_load(A + ((long long)col * nb + row) * 64);
  };
  // forward, in place: y_i = (P r)_i - sum_{j<i} L_ij y_j
  for (int i0 = 0; i0 < nb; i0 += RB) {
    const int nr = nb - i0 < RB ? nb - i0 : RB;
    F acc[RB];
#pragma unroll
    for (int q = 0; q < RB; ++q) acc[q] = ys[(i0 + (q < nr ? q : nr - 1)) * 64 + lane];
#pragma unroll 2
    for (int j = 0; j < i0; ++j) {
      const F yj = ys[j * 64 + lane];
#pragma unroll
      for (int q = 0; q < RB; ++q) acc[q] -= entry(i0 + q, j) * yj;
    }
#pragma unroll
    for (int q = 1; q < RB; ++q)
#pragma unroll
      for (int c = 0; c < q; ++c) acc[q] -= entry(i0 + q, i0 + c) * acc[c];
#pragma unroll
    for (int q = 0; q < RB; ++q)
      if (q < nr) ys[(i0 + q) * 64 + lane] = acc[q];
  }
  // backward: z_i = (y_i - sum_{j>i} U_ij z_j) / U_ii, in place over y
  for (int i1 = nb; i1 > 0; i1 -= RB) {
    const int i0 = i1 - RB > 0 ? i1 - RB : 0;
    const int nr = i1 - i0;
    F acc[RB];
#pragma unroll
    for (int q = 0; q < RB; ++q) acc[q] = ys[(i0 + (q < nr ? q : nr - 1)) * 64 + lane];
#pragma unroll 2
    for (int j = i1; j < nb; ++j) {
      const F zj = ys[j * 64 + lane];
#pragma unroll
      for (int q = 0; q < RB; ++q) acc[q] -= entry(i0 + q, j) * zj;
    }
#pragma unroll
    for (int q = 0; q < RB; ++q) acc[q] = q < nr ? acc[q] : F(0);   // rows past the chunk: 0
#pragma unroll
    for (int q = RB - 1; q >= 0; --q) {
#pragma unroll
      for (int c = q + 1; c < RB; ++c) acc[q] -= entry(i0 + q, i0 + c) * acc[c];
      acc[q] = q < nr ? acc[q] / entry(i0 + q, i0 + q) : F(0);
    }
#pragma unroll
    for (int q = 0; q < RB; ++q)
      if (q < nr) ys[(i0 + q) * 64 + lane] = acc[q];
  }
  if (!valid) return;
  for (int l = 0; l < nb; ++l) {
    bool wall;
    const long long d = block_dof(L, b, l, wall);
    zz[d] = wall ? R(0) : (R)ys[l * 64 + lane];
  }
}

BLayout layout_of(const Ctx* c) {
  BLayout L{};
  L.nv = c->nv;
  L.nx = c->op.nx;
  L.ny = c->op.ny;
  L.nz = c->op.nz;
  L.bx = c->pc_bx;
  L.by = c->pc_by;
  L.bz = c->pc_bz;
  L.nbx = L.nx / L.bx;
  L.nby = L.ny / L.by;
  L.nbz = L.nz / L.bz;
  L.cells = L.bx * L.by * L.bz;
  L.nb = L.nv * L.cells;
  L.nblocks = (long long)L.nbx * L.nby * L.nbz;
  L.npts = c->op.npts;
  L.bcy = c->op.bcy;
  return L;
}

int colours(int nblk, int width, bool periodic, int ndim_ok) {
  if (!ndim_ok || nblk == 1) return 1;
  int cnum = 1 + (3 + width - 1) / width;
  if (cnum > nblk) cnum = nblk;
  if (periodic && nblk % cnum) return -1;
  return cnum;
}

inline unsigned blocks_for(long long n, int threads) { return (unsigned)((n + threads - 1) / threads); }

}  // namespace

template <typename R>
hipError_t precond_apply(Ctx* c, int ishift, int nrhs, const R* r, R* z, const int* active, int shift_step,
                         long long sV, long long sA, hipStream_t s) {
  if (c->pc_kind == SA_PC_MEAN_FLOW) return fourier_apply<R>(c, ishift, nrhs, r, z, active, shift_step, sV, sA, s);
  BLayout L = layout_of(c);
  dim3 grid((unsigned)((L.nblocks + 63) / 64), (unsigned)nrhs);
  if (sV == 0) sV = c->n;
  if (c->pc_f64)
    apply_kernel<double, R><<<grid, 64, sizeof(double) * L.nb * 64, s>>>(
        L, (const double*)c->pc_lu, c->pc_perm, ishift, shift_step, r, z, sV, active, sA);
  else
    apply_kernel<float, R><<<grid, 64, sizeof(float) * L.nb * 64, s>>>(
        L, (const float*)c->pc_lu, c->pc_perm, ishift, shift_step, r, z, sV, active, sA);
  return hipGetLastError();
}
template hipError_t precond_apply<double>(Ctx*, int, int, const double*, double*, const int*, int, long long,
                                          long long, hipStream_t);
template hipError_t precond_apply<float>(Ctx*, int, int, const float*, float*, const int*, int, long long,
                                         long long, hipStream_t);

}  // namespace sa

using namespace sa;

extern "C" int sa_precond_setup(sa_ctx* c, const sa_precond_opts* o, int nshift, const double* shifts_host) {
  if (!c) return SA_EINVAL;
  if (!c->has_base) return c->fail(SA_ESTATE, "sa_precond_setup: call sa_base_set first");
  if (!o || !shifts_host || nshift < 1) return c->fail(SA_EINVAL, "sa_precond_setup: null argument or nshift < 1");
  if (o->kind != SA_PC_BLOCK_JACOBI && o->kind != SA_PC_MEAN_FLOW)
    return c->fail(SA_EINVAL, "sa_precond_setup: bad preconditioner kind %d", o->kind);
  if (o->kind == SA_PC_MEAN_FLOW) {
    c->has_precond = false;
    c->drop_graphs();
    const int rc = fourier_setup(c, o, nshift, shifts_host);
    if (rc != SA_OK) return rc;
    c->pc_kind = SA_PC_MEAN_FLOW;
    c->pc_nshift = nshift;
    c->has_precond = true;
    return SA_OK;
  }
  const int bz = c->op.ndim == 2 ? 1 : o->bz;
  if (o->bx < 1 || o->by < 1 || bz < 1) return c->fail(SA_EINVAL, "sa_precond_setup: bad block size");
  if (c->op.nx % o->bx || c->op.ny % o->by || c->op.nz % bz)
    return c->fail(SA_EINVAL, "sa_precond_setup: grid not divisible by the block size");
  if (o->factor_prec != SA_F32 && o->factor_prec != SA_F64)
    return c->fail(SA_EINVAL, "sa_precond_setup: factor precision must be SA_F32 or SA_F64");
  c->has_precond = false;
  c->drop_graphs();
  c->pc_bx = o->bx;
  c->pc_by = o->by;
  c->pc_bz = bz;
  BLayout L = layout_of(c);
  if (L.nb > 128) return c->fail(SA_EINVAL, "sa_precond_setup: block order %d exceeds 128", L.nb);
  if (o->factor_prec == SA_F64 && L.nb > 90)
    return c->fail(SA_EINVAL, "sa_precond_setup: FP64 factors need block order <= 90");
  const int cx = colours(L.nbx, L.bx, true, 1);
  const int cy = colours(L.nby, L.by, c->op.bcy == 0, 1);
  const int cz = colours(L.nbz, L.bz, true, c->op.ndim == 3);
  if (cx < 0 || cy < 0 || cz < 0)
    return c->fail(SA_EINVAL, "sa_precond_setup: periodic block count not divisible by the probe colour count");
  hipStream_t s = c->stream;
  const long long n = c->n;
  const size_t bbytes = sizeof(double) * (size_t)L.nblocks * L.nb * L.nb;
  double* B = (double*)c->buffer("pc_B", bbytes);
  double* sh = (double*)c->buffer("pc_shifts", sizeof(double) * nshift, false);
  int* flag = (int*)c->buffer("flag", sizeof(int));
  const size_t fsz = o->factor_prec == SA_F64 ? sizeof(double) : sizeof(float);
  const size_t padded = (size_t)((L.nblocks + 63) / 64) * 64;   // blocks, interleaved in groups of 64
  void* LU = c->buffer("pc_LU", fsz * (size_t)nshift * padded * L.nb * L.nb, false);
  int* perm = (int*)c->buffer("pc_perm", sizeof(int) * (size_t)nshift * padded * L.nb, false);
  // probes in the factor precision: FP32 factors take blocks probed with the
  // FP32 operator (half the bytes of the FP64 one)
  const int batch = L.nb < 16 ? L.nb : 16;
  void* E = c->buffer("pc_probe", fsz * n * batch, false);
  void* Y = c->buffer("pc_resp", fsz * n * batch, false);
  if (!B || !sh || !flag || !LU || !perm || !E || !Y) return c->fail(SA_ENOMEM, "sa_precond_setup: out of device memory");
  hipMemsetAsync(E, 0, fsz * n * batch, s);   // once: each probe batch resets its own entries
  hipMemsetAsync(B, 0, bbytes, s);
  hipMemcpyAsync(sh, shifts_host, sizeof(double) * nshift, hipMemcpyHostToDevice, s);
  auto probe = [&](auto one) -> hipError_t {
    using F = decltype(one);
    F* Ef = static_cast<F*>(E);
    F* Yf = static_cast<F*>(Y);
    const int ncol = cx * cy * cz;
    for (int col = 0; col < ncol; ++col) {
      const ColourSet q = colour_set(L, col, cx, cy, cz);
      if (q.count == 0) continue;
      for (int l0 = 0; l0 < L.nb; l0 += batch) {
        const int np = std::min(batch, L.nb - l0);
        const unsigned gf = blocks_for(q.count * np, 256);
        probe_fill_kernel<F><<<gf, 256, 0, s>>>(L, q, Ef, n, cx, cy, cz, l0, np, one);
        hipError_t e = c->jv<F>(Ef, Yf, np, 0.0, nullptr);
        if (e != hipSuccess) return e;
        probe_extract_kernel<F><<<blocks_for(q.count * L.nb * np, 256), 256, 0, s>>>(L, q, Yf, n, B, cx, cy, cz, l0,
                                                                                    np);
        probe_fill_kernel<F><<<gf, 256, 0, s>>>(L, q, Ef, n, cx, cy, cz, l0, np, F(0));
      }
    }
    return hipGetLastError();
  };
  {
    const hipError_t e = o->factor_prec == SA_F64 ? probe(1.0) : probe(1.0f);
    if (e != hipSuccess) return c->hip_fail(e, "sa_precond_setup probe");
  }
  if (o->noise_std != 0.0)
    add_noise_kernel<<<blocks_for(L.nblocks * L.nb * L.nb, 256), 256, 0, s>>>(L, B, o->noise_std, o->seed);
  hipMemsetAsync(flag, 0, sizeof(int), s);
  const size_t lds = fsz * L.nb * L.nb;
  if ((long long)L.nblocks * nshift >= (1LL << 31)) return c->fail(SA_EINVAL, "sa_precond_setup: too many blocks");
  const unsigned grid = (unsigned)(L.nblocks * nshift);
  if (o->factor_prec == SA_F64)
    lu_kernel<double><<<grid, 256, lds, s>>>(L, B, sh, o->diag_add, (double*)LU, perm, flag);
  else if (L.nb % 16 == 0)   // LDS block with leading dimension nb + 1
    lu_mfma_kernel<<<grid, LU_MFMA_THREADS, sizeof(float) * L.nb * (L.nb + 1), s>>>(L, B, sh, o->diag_add,
                                                                                      (float*)LU, perm, flag);
  else
    lu_kernel<float><<<grid, 256, lds, s>>>(L, B, sh, o->diag_add, (float*)LU, perm, flag);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return c->hip_fail(e, "sa_precond_setup factor");
  int hflag = 0;
  hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s);
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return c->hip_fail(e, "sa_precond_setup sync");
  if (hflag) return c->fail(SA_ESINGULAR, "sa_precond_setup: zero pivot in a block");
  c->pc_lu = LU;
  c->pc_perm = perm;
  c->pc_f64 = o->factor_prec == SA_F64;
  c->pc_kind = SA_PC_BLOCK_JACOBI;
  c->pc_nshift = nshift;
  c->pc_nb = L.nb;
  c->pc_nblocks = L.nblocks;
  c->has_precond = true;
  return SA_OK;
}

extern "C" int sa_precond_apply(sa_ctx* c, sa_prec prec, int ishift, int nrhs, const void* r_dev, void* z_dev) {
  if (!c) return SA_EINVAL;
  if (!c->has_precond) return c->fail(SA_ESTATE, "sa_precond_apply: call sa_precond_setup first");
  if (ishift < 0 || ishift >= c->pc_nshift || nrhs < 1 || !r_dev || !z_dev)
    return c->fail(SA_EINVAL, "sa_precond_apply: bad shift index, nrhs or pointer");
  if (c->pc_kind == SA_PC_MEAN_FLOW && nrhs > c->fp_nrhs_cap)
    return c->fail(SA_EINVAL, "sa_precond_apply: the mean-flow preconditioner takes at most %d vectors per call",
                   c->fp_nrhs_cap);
  hipError_t e;
  if (prec == SA_F64)
    e = precond_apply<double>(c, ishift, nrhs, (const double*)r_dev, (double*)z_dev, nullptr, 0, 0, 0, c->stream);
  else if (prec == SA_F32)
    e = precond_apply<float>(c, ishift, nrhs, (const float*)r_dev, (float*)z_dev, nullptr, 0, 0, 0, c->stream);
  else
    return c->fail(SA_EINVAL, "sa_precond_apply: precision must be SA_F64 or SA_F32");
  if (e != hipSuccess) return c->hip_fail(e, "sa_precond_apply");
  return SA_OK;
}

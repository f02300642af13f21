// Vector kernels of the Krylov solvers: multi-dot products against a block of
// basis vectors, the fused Gram-Schmidt update w += s V h with the next pass's
// dot products, norms, scaling and precision casts.
//
// Every reduction is deterministic: a fixed number of blocks (a function of
// n only) writes one partial per block and per column in double precision,
// and the partials are summed in a fixed order, by a second kernel or, for
// up to FUSE_MAX_BLOCKS blocks, by the last block of the reducing kernel to
// finish (arrival counter); GMRES's Arnoldi step then runs in that block too.  All kernels take
// an `active` device flag and return at once when it is zero, so that a whole
// GMRES cycle can be enqueued ahead and stop on the device when it converges.
// A batch of independent systems runs in one launch: blockIdx.z (blockIdx.y
// for the reductions) is the system, with the strides of a Batch.
#include "blas.h"

namespace sa {
namespace {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

__device__ __forceinline__ bool inactive(const int* active, long long sA) {
  return active && !active[blockIdx.z * sA];
}

// E consecutive elements moved by one load / store (E = 16 / sizeof(R) on
// the 16-byte path, 1 on the scalar path); NT: nontemporal (data streamed
// once, kept from displacing what is re-read).
template <typename R, int E, bool NT = false>
__device__ __forceinline__ void vload(const R* p, R (&v)[E]) {
  if constexpr (E == 1) {
    v[0] = NT ? __builtin_nontemporal_load(p) : *p;
  } else {
    typedef R vt __attribute__((ext_vector_type(E)));
    const vt* q = reinterpret_cast<const vt*>(p);
    const vt x = NT ? __builtin_nontemporal_load(q) : *q;
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = x[e];
  }
}
template <typename R, int E>
__device__ __forceinline__ void vstore(R* p, const R (&v)[E]) {
  if constexpr (E == 1) {
    *p = v[0];
  } else {
    typedef R vt __attribute__((ext_vector_type(E)));
    vt x;
#pragma unroll
    for (int e = 0; e < E; ++e) x[e] = v[e];
    *reinterpret_cast<vt*>(p) = x;
  }
}

// Sum acc[c] over the block for c < ncol; writes out[c].
template <int MAXC>
__device__ __forceinline__ void block_sum_cols(double (&acc)[MAXC], int ncol, double* __restrict__ out) {
  __shared__ double red[RED_THREADS / 64][MAXC];
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < MAXC; ++c) {
    if (c < ncol) {
      const double s = wave_sum(acc[c]);
      if (lane == 0) red[wid][c] = s;
    }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < ncol; c += blockDim.x) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < RED_THREADS / 64; ++w) s += red[w][c];
    out[c] = s;
  }
}

// Where a reduction ends: out[c] (+)= sum over the partials of the system.
// With a ticket, the last block of the system to arrive does the sum (fixed
// order over blocks and lanes, so deterministic) and, for a GMRES state,
// the Arnoldi step that consumes it.
struct RedEnd {
  double* out;
  long long sR;     // out stride between systems (doubles)
  int accumulate;
  int* ticket;      // per system arrival counter (zero between launches), or null
  GState* step;     // GMRES states (stride sR doubles), or null
  int step_j;
};

// nblk partial rows; narrive blocks of the system take part (all write
// their partials before arriving).
__device__ __forceinline__ void finish_reduction(const double* __restrict__ partial, int nblk, int narrive, int ldp,
                                                 int ncol, const RedEnd& e) {
  if (!e.ticket) return;
  const long long sys = blockIdx.z;
  __shared__ int is_last;
  __syncthreads();   // this block's partials are written
  if (threadIdx.x == 0) {
    __threadfence();
    const int t = atomicAdd(e.ticket + sys, 1);
    is_last = t == narrive - 1;
    if (is_last) atomicExch(e.ticket + sys, 0);
  }
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  double* out = e.out + sys * e.sR;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int c = wid; c < ncol; c += RED_THREADS / 64) {
    double s = 0.0;
    for (int b = lane; b < nblk; b += 64) s += partial[(long long)b * ldp + c];
    s = wave_sum(s);
    if (lane == 0) out[c] = e.accumulate ? out[c] + s : s;
  }
  if (e.step) {
    __syncthreads();
    __threadfence_block();
    gstate_step_block(reinterpret_cast<GState*>(reinterpret_cast<double*>(e.step) + sys * e.sR), e.step_j);
  }
}

// partial[b*ldp + c0 + c] = sum over this block's elements of V[c0+c][i] w[i]
// (blockIdx.y: column chunk, blockIdx.z: system); threads take E elements at
// a time (n, ldv and the strides are multiples of E)
template <typename R, int MAXC, int E, bool NT>
__global__ void __launch_bounds__(RED_THREADS) multidot_kernel(long long n, const R* __restrict__ V, long long ldv,
                                                               int ncol, const R* __restrict__ w,
                                                               double* __restrict__ partial, int ldp,
                                                               const int* __restrict__ active, long long sV,
                                                               long long sP, long long sA, RedEnd e) {
  if (inactive(active, sA)) return;
  const long long sys = blockIdx.z;
  V += sys * sV;
  w += sys * sV;
  partial += sys * sP;
  const int c0 = blockIdx.y * MAXC;
  const int nc = min(MAXC, ncol - c0);
  double acc[MAXC];
#pragma unroll
  for (int c = 0; c < MAXC; ++c) acc[c] = 0.0;
  const long long nch = n / E;
  const long long stride = (long long)gridDim.x * blockDim.x;
#pragma unroll 1
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < nch; k += stride) {
    R wv[E];
    vload<R, E>(w + k * E, wv);
#pragma unroll
    for (int c = 0; c < MAXC; ++c)
      if (c < nc) {
        R v[E];
        vload<R, E, NT>(V + (long long)(c0 + c) * ldv + k * E, v);
        double t = (double)v[0] * (double)wv[0];
#pragma unroll
        for (int q = 1; q < E; ++q) t += (double)v[q] * (double)wv[q];
        acc[c] += t;
      }
  }
  block_sum_cols<MAXC>(acc, nc, partial + (long long)blockIdx.x * ldp + c0);
  finish_reduction(partial, gridDim.x, gridDim.x * gridDim.y, ldp, ncol, e);
}

// w_new = w + hsign * sum_c V[c] h[c]; writes w_new to wout (may alias w).
// norm: partial ||w_new||^2 in column 0.  The coefficients sit in LDS.
// Columns after the last non-zero coefficient are not read: a GMRES cycle
// that ends early leaves its later basis columns unwritten (stale, possibly
// non-finite), and its solution update passes zeros for them.
template <typename R, int MAXC, int E, bool NT>
__global__ void __launch_bounds__(RED_THREADS) update_kernel(
    long long n, const R* __restrict__ V, long long ldv, int ncol, const double* __restrict__ h, double hsign,
    const R* w, R* wout, int norm, double* __restrict__ partial, int ldp, const int* __restrict__ active,
    long long sV, long long sR, long long sP, long long sA, long long sW, RedEnd e) {
  if (inactive(active, sA)) return;
  const long long sys = blockIdx.z;
  V += sys * sV;
  w += sys * sW;
  wout += sys * sW;
  h += sys * sR;
  partial += sys * sP;
  __shared__ double hc[MAXC];
  __shared__ int s_nc;
  for (int c = threadIdx.x; c < MAXC; c += blockDim.x) hc[c] = c < ncol ? hsign * h[c] : 0.0;
  __syncthreads();
  if (threadIdx.x == 0) {
    int last = 0;
    for (int c = 0; c < ncol; ++c)
      if (hc[c] != 0.0) last = c + 1;
    s_nc = last;
  }
  __syncthreads();
  const int nc = s_nc;
  double acc[1] = {0.0};
  const long long nch = n / E;
  const long long stride = (long long)gridDim.x * blockDim.x;
#pragma unroll 1
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < nch; k += stride) {
    R wv[E];
    vload<R, E>(w + k * E, wv);
    double sum[E];
#pragma unroll
    for (int q = 0; q < E; ++q) sum[q] = (double)wv[q];
#pragma unroll 8
    for (int c = 0; c < nc; ++c) {
      R v[E];
      vload<R, E, NT>(V + (long long)c * ldv + k * E, v);
#pragma unroll
      for (int q = 0; q < E; ++q) sum[q] += (double)v[q] * hc[c];
    }
    R wn[E];
#pragma unroll
    for (int q = 0; q < E; ++q) {
      wn[q] = (R)sum[q];
      acc[0] += (double)wn[q] * (double)wn[q];
    }
    vstore<R, E>(wout + k * E, wn);
  }
  if (!norm) return;
  block_sum_cols<1>(acc, 1, partial + (long long)blockIdx.x * ldp);
  finish_reduction(partial, gridDim.x, gridDim.x, ldp, 1, e);
}

// The same update followed by the dots V^T w_new (partial per block and
// column), reading V once.  The four 16-lane groups of a wave share 16
// chunks of E elements: group g holds columns g, g + 4, ... (KC of them) of
// its chunk in registers, the groups' partial sums of V h are combined with
// two xor shuffles (the same fixed order on all four lanes, so they agree
// bit for bit), group 0 stores w_new, and each group accumulates the dots of
// its own columns.  Lanes whose last column lies past ncol read column
// ncol - 1 again (a cached duplicate) with coefficient 0, so every load is
// unconditional.
template <typename R, int KC, int E, bool NT>
__global__ void __launch_bounds__(RED_THREADS) update_dot_kernel(
    long long n, const R* __restrict__ V, long long ldv, int ncol, const double* __restrict__ h, double hsign,
    const R* w, R* wout, double* __restrict__ partial, int ldp, const int* __restrict__ active, long long sV,
    long long sR, long long sP, long long sA, long long sW, RedEnd e) {
  constexpr int NG = 4;
  constexpr int NW = RED_THREADS / 64;
  constexpr int MAXC = NG * KC;
  if (inactive(active, sA)) return;
  const long long sys = blockIdx.z;
  V += sys * sV;
  w += sys * sW;
  wout += sys * sW;
  h += sys * sR;
  partial += sys * sP;
  __shared__ double hc[MAXC];
  __shared__ double red[NW][MAXC];
  for (int c = threadIdx.x; c < MAXC; c += blockDim.x) hc[c] = c < ncol ? hsign * h[c] : 0.0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int g = lane >> 4, sl = lane & 15;
  const R* Vk[KC];
  double hk[KC];
#pragma unroll
  for (int k = 0; k < KC; ++k) {
    const int c = g + NG * k;
    Vk[k] = V + (long long)(c < ncol ? c : ncol - 1) * ldv;
    hk[k] = hc[c];
  }
  double acc[KC];
#pragma unroll
  for (int k = 0; k < KC; ++k) acc[k] = 0.0;
  const long long nch = n / E;
  const long long cstride = (long long)gridDim.x * NW * 16;
#pragma unroll 1
  for (long long q0 = ((long long)blockIdx.x * NW + wid) * 16 + sl; q0 < nch; q0 += cstride) {
    const long long i = q0 * E;
    R v[KC][E];
#pragma unroll
    for (int k = 0; k < KC; ++k) vload<R, E, NT>(Vk[k] + i, v[k]);
    R wv[E];
    vload<R, E>(w + i, wv);
    double p[E];
#pragma unroll
    for (int q = 0; q < E; ++q) {
      double t = 0.0;
#pragma unroll
      for (int k = 0; k < KC; ++k) t += (double)v[k][q] * hk[k];
      t += __shfl_xor(t, 16, 64);
      t += __shfl_xor(t, 32, 64);
      p[q] = t;
    }
    R wn[E];
#pragma unroll
    for (int q = 0; q < E; ++q) wn[q] = (R)((double)wv[q] + p[q]);
    if (g == 0) vstore<R, E>(wout + i, wn);
#pragma unroll
    for (int k = 0; k < KC; ++k) {
      double t = (double)v[k][0] * (double)wn[0];
#pragma unroll
      for (int q = 1; q < E; ++q) t += (double)v[k][q] * (double)wn[q];
      acc[k] += t;
    }
  }
  // per column: sum over the 16 lanes of its group, then over the waves
#pragma unroll
  for (int k = 0; k < KC; ++k) {
    double t = acc[k];
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) t += __shfl_down(t, off, 16);
    if (sl == 0) red[wid][g + NG * k] = t;
  }
  __syncthreads();
  double* prow = partial + (long long)blockIdx.x * ldp;
  for (int c = threadIdx.x; c < ncol; c += blockDim.x) {
    double t = red[0][c];
#pragma unroll
    for (int q = 1; q < NW; ++q) t += red[q][c];
    prow[c] = t;
  }
  finish_reduction(partial, gridDim.x, gridDim.x, ldp, ncol, e);
}

// out[c] = (accumulate ? out[c] : 0) + sum_b partial[b*ldp + c]  (fixed order)
// blockIdx.x: column, blockIdx.y: system
__global__ void reduce_cols_kernel(const double* __restrict__ partial, int nblocks, int ldp, int ncol,
                                   double* __restrict__ out, int accumulate, const int* __restrict__ active,
                                   long long sR, long long sP, long long sA) {
  const long long sys = blockIdx.y;
  if (active && !active[sys * sA]) return;
  partial += sys * sP;
  out += sys * sR;
  const int c = blockIdx.x;
  if (c >= ncol) return;
  __shared__ double red[RED_THREADS];
  double s = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x) s += partial[(long long)b * ldp + c];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[c] = accumulate ? out[c] + red[0] : red[0];
}

// partial ||x||^2 (column 0)
template <typename R>
__global__ void __launch_bounds__(RED_THREADS) nrm2_kernel(long long n, const R* __restrict__ x,
                                                           double* __restrict__ partial, int ldp,
                                                           const int* __restrict__ active, long long sV,
                                                           long long sP, long long sA, RedEnd e) {
  if (inactive(active, sA)) return;
  x += blockIdx.z * sV;
  partial += blockIdx.z * sP;
  double acc[1] = {0.0};
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double v = (double)x[i];
    acc[0] += v * v;
  }
  block_sum_cols<1>(acc, 1, partial + (long long)blockIdx.x * ldp);
  finish_reduction(partial, gridDim.x, gridDim.x, ldp, 1, e);
}

// r = b - y, partial ||r||^2 (b uses its own stride sB; y null: y = 0)
template <typename R>
__global__ void __launch_bounds__(RED_THREADS) residual_kernel(long long n, const R* __restrict__ b,
                                                               const R* __restrict__ y, R* __restrict__ r,
                                                               double* __restrict__ partial, int ldp,
                                                               const int* __restrict__ active, long long sV,
                                                               long long sB, long long sP, long long sA,
                                                               long long sY, RedEnd e) {
  if (inactive(active, sA)) return;
  const bool hy = y != nullptr;
  b += blockIdx.z * sB;
  if (hy) y += blockIdx.z * sY;
  r += blockIdx.z * sV;
  partial += blockIdx.z * sP;
  double acc[1] = {0.0};
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const R v = hy ? b[i] - y[i] : b[i];
    r[i] = v;
    acc[0] += (double)v * (double)v;
  }
  block_sum_cols<1>(acc, 1, partial + (long long)blockIdx.x * ldp);
  finish_reduction(partial, gridDim.x, gridDim.x, ldp, 1, e);
}

// out = x * (*scale)   (scale read from device memory)
template <typename R, int E>
__global__ void scale_kernel(long long n, const R* x, R* out, const double* __restrict__ scale,
                             const int* __restrict__ active, long long sV, long long sR, long long sA) {
  if (inactive(active, sA)) return;
  x += blockIdx.z * sV;
  out += blockIdx.z * sV;
  const double a = scale[blockIdx.z * sR];
  const long long nch = n / E;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < nch; k += stride) {
    R v[E];
    vload<R, E>(x + k * E, v);
#pragma unroll
    for (int q = 0; q < E; ++q) v[q] = (R)((double)v[q] * a);
    vstore<R, E>(out + k * E, v);
  }
}

// out = (To)(x * (*scale)) with a precision change
template <typename Ti, typename To>
__global__ void cast_scale_kernel(long long n, const Ti* __restrict__ x, To* __restrict__ out,
                                  const double* __restrict__ scale, int accumulate) {
  const double a = scale ? *scale : 1.0;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double v = (double)x[i] * a;
    out[i] = accumulate ? (To)((double)out[i] + v) : (To)v;
  }
}

template <typename R>
__global__ void lincomb_kernel(long long n, const R* x, long long sx, double a, const R* y, long long sy, double c,
                               R* out, long long so, const int* __restrict__ active, long long sA) {
  if (inactive(active, sA)) return;
  x += blockIdx.z * sx;
  y += blockIdx.z * sy;
  out += blockIdx.z * so;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    out[i] = (R)(a * (double)x[i] + c * (double)y[i]);
}

template <typename R>
__global__ void fill_kernel(long long n, R* __restrict__ x, R v) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) x[i] = v;
}

inline unsigned grid_for(long long n) {
  long long b = (n + RED_THREADS - 1) / RED_THREADS;
  if (b > RED_BLOCKS) b = RED_BLOCKS;
  if (b < 1) b = 1;
  return (unsigned)b;
}

inline long long part_stride(int ldp) { return (long long)RED_BLOCKS * ldp; }

// Blocks for nch chunks (one per thread and grid step).  Mid-size vectors
// that would leave compute units idle get two blocks per unit (at least 64
// chunks each), which measured faster than one block per unit with the
// reduction finished in the kernel; short vectors keep few blocks (latency).
constexpr int NUM_CU = 256;
inline unsigned grid_for_chunks(long long nch) {
  const unsigned b = grid_for(nch);
  if (b < (unsigned)NUM_CU && nch >= 128ll * NUM_CU) return 2 * NUM_CU;
  return b;
}

// Chunk width of the vector kernels: 16-byte loads when every column, vector
// and system stride allows it, else one element.
template <typename R>
int chunk_width(long long n, long long ldv, const Batch& b, const void* p0, const void* p1 = nullptr,
                const void* p2 = nullptr) {
  constexpr int E = 16 / sizeof(R);
  if (n % E || ldv % E || b.vec % E || b.w() % E) return 1;
  for (const void* p : {p0, p1, p2})
    if (reinterpret_cast<uintptr_t>(p) % 16) return 1;
  return E;
}

// Basis columns of at least this many bytes are streamed with nontemporal
// loads in the single-pass kernels (they are not re-read from cache before
// the next pass anyway).
constexpr long long NT_MIN_BYTES = 4ll << 20;

}  // namespace

template <typename R>
RedEnd reduction_end(const Blas<R>& bl, unsigned nb, double* out, bool accumulate, const Batch& b,
                     GState* step = nullptr, int step_j = 0) {
  const bool fused = bl.ticket && nb <= (unsigned)FUSE_MAX_BLOCKS;
  return RedEnd{out, b.res, accumulate ? 1 : 0, fused ? bl.ticket : nullptr, fused ? step : nullptr, step_j};
}

template <typename R>
void Blas<R>::multidot(long long n, const R* V, long long ldv, int ncol, const R* w, double* out, bool accumulate,
                       const int* active, hipStream_t s, const Batch& b) const {
  constexpr int VE = 16 / sizeof(R);
  const int E = chunk_width<R>(n, ldv, b, V, w);
  const bool nt = n * (long long)sizeof(R) >= NT_MIN_BYTES;
  const int chunks = (ncol + 15) / 16;
  const unsigned nb = grid_for_chunks(n / E);
  const long long sP = part_stride(ldp);
  const RedEnd e = reduction_end(*this, nb, out, accumulate, b);
  const dim3 grid(nb, chunks, b.nsys);
#define SA_MULTIDOT(EE, NT)                                                                                        \
  multidot_kernel<R, 16, EE, NT><<<grid, RED_THREADS, 0, s>>>(n, V, ldv, ncol, w, partial, ldp, active, b.vec, sP, \
                                                             b.act, e)
  if (E == VE) {
    if (nt) SA_MULTIDOT(VE, true); else SA_MULTIDOT(VE, false);
  } else {
    if (nt) SA_MULTIDOT(1, true); else SA_MULTIDOT(1, false);
  }
#undef SA_MULTIDOT
  if (!e.ticket)
    reduce_cols_kernel<<<dim3(ncol, b.nsys), RED_THREADS, 0, s>>>(partial, (int)nb, ldp, ncol, out,
                                                                  accumulate ? 1 : 0, active, b.res, sP, b.act);
}

template <typename R>
bool Blas<R>::update(long long n, const R* V, long long ldv, int ncol, const double* h, double hsign, const R* w,
                     R* wout, int mode, double* out, bool accumulate, const int* active, hipStream_t s,
                     const Batch& b, GState* step, int step_j) const {
  // mode: 0 = no reduction, 1 = dots V^T w_new, 2 = ||w_new||^2
  constexpr int CH = 48;   // columns per launch
  constexpr int VE = 16 / sizeof(R);
  const bool dot = mode == 1;
  const int E = chunk_width<R>(n, ldv, b, V, w, wout);
  const bool nt = n * (long long)sizeof(R) >= NT_MIN_BYTES;
  const unsigned nb = grid_for_chunks(n / E);
  const long long sP = part_stride(ldp);
  const dim3 grid(nb, 1, b.nsys);
  const RedEnd none{nullptr, 0, 0, nullptr, nullptr, 0};
  const RedEnd e = reduction_end(*this, nb, out, accumulate, b, mode == 2 ? step : nullptr, step_j);
  int done = 0;
  const R* src = w;
  bool reduced = false;   // the reduction ran inside the last launch
  unsigned nb_dot = nb;   // partial rows of the dot reduction
  for (;;) {
    const int c = ncol - done < CH ? ncol - done : CH;
    const bool last = done + c >= ncol;
    const R* Vc = V + (long long)done * ldv;
    if (last && dot && ncol <= CH) {
      // 16 chunks per wave and grid step: its own block count and reduction
      const unsigned nbd = grid_for(4 * (n / E));
      const RedEnd ed = reduction_end(*this, nbd, out, accumulate, b);
      const dim3 gridd(nbd, 1, b.nsys);
      nb_dot = nbd;
#define SA_UPDOT(KC, EE, NT)                                                                                    \
  update_dot_kernel<R, KC, EE, NT><<<gridd, RED_THREADS, 0, s>>>(n, Vc, ldv, c, h + done, hsign, src, wout, partial, \
                                                                 ldp, active, b.vec, b.res, sP, b.act, b.w(), ed)
#define SA_UPDOT_E(KC) \
  if (E != VE) SA_UPDOT(KC, 1, false); else if (nt) SA_UPDOT(KC, VE, true); else SA_UPDOT(KC, VE, false)
      switch ((c + 3) / 4) {
        case 1: SA_UPDOT_E(1); break;
        case 2: SA_UPDOT_E(2); break;
        case 3: SA_UPDOT_E(3); break;
        case 4: SA_UPDOT_E(4); break;
        case 5: SA_UPDOT_E(5); break;
        case 6: SA_UPDOT_E(6); break;
        case 7: SA_UPDOT_E(7); break;
        case 8: SA_UPDOT_E(8); break;
        case 9: SA_UPDOT_E(9); break;
        case 10: SA_UPDOT_E(10); break;
        case 11: SA_UPDOT_E(11); break;
        default: SA_UPDOT_E(12); break;
      }
#undef SA_UPDOT_E
#undef SA_UPDOT
      reduced = ed.ticket != nullptr;
    } else {
      const int norm = last && mode == 2 ? 1 : 0;
      const RedEnd& ee = norm ? e : none;
#define SA_UPD(MC, EE, NT)                                                                                        \
  update_kernel<R, MC, EE, NT><<<grid, RED_THREADS, 0, s>>>(n, Vc, ldv, c, h + done, hsign, src, wout, norm, partial, \
                                                            ldp, active, b.vec, b.res, sP, b.act, b.w(), ee)
      if (c <= 16) {
        if (E == VE) { if (nt) SA_UPD(16, VE, true); else SA_UPD(16, VE, false); }
        else { if (nt) SA_UPD(16, 1, true); else SA_UPD(16, 1, false); }
      } else {
        if (E == VE) { if (nt) SA_UPD(CH, VE, true); else SA_UPD(CH, VE, false); }
        else { if (nt) SA_UPD(CH, 1, true); else SA_UPD(CH, 1, false); }
      }
#undef SA_UPD
      reduced = norm && e.ticket != nullptr;
    }
    src = wout;
    done += c;
    if (last) break;
  }
  if (dot && ncol > CH) {
    multidot(n, V, ldv, ncol, wout, out, accumulate, active, s, b);
  } else if (mode == 1 && !reduced) {
    reduce_cols_kernel<<<dim3(ncol, b.nsys), RED_THREADS, 0, s>>>(partial, (int)nb_dot, ldp, ncol, out,
                                                                  accumulate ? 1 : 0, active, b.res, sP, b.act);
  } else if (mode == 2 && !reduced) {
    reduce_cols_kernel<<<dim3(1, b.nsys), RED_THREADS, 0, s>>>(partial, (int)nb, ldp, 1, out, accumulate ? 1 : 0,
                                                               active, b.res, sP, b.act);
  }
  return mode == 2 && step && reduced;
}

template <typename R>
void Blas<R>::nrm2sq(long long n, const R* x, double* out, const int* active, hipStream_t s, const Batch& b) const {
  const unsigned nb = grid_for(n);
  const long long sP = part_stride(ldp);
  const RedEnd e = reduction_end(*this, nb, out, false, b);
  nrm2_kernel<R><<<dim3(nb, 1, b.nsys), RED_THREADS, 0, s>>>(n, x, partial, ldp, active, b.vec, sP, b.act, e);
  if (!e.ticket)
    reduce_cols_kernel<<<dim3(1, b.nsys), RED_THREADS, 0, s>>>(partial, (int)nb, ldp, 1, out, 0, active, b.res, sP,
                                                               b.act);
}

template <typename R>
void Blas<R>::residual(long long n, const R* bvec, const R* y, R* r, double* out, const int* active, hipStream_t s,
                       const Batch& b, long long sB, long long sY) const {
  const unsigned nb = grid_for(n);
  const long long sP = part_stride(ldp);
  const RedEnd e = reduction_end(*this, nb, out, false, b);
  residual_kernel<R><<<dim3(nb, 1, b.nsys), RED_THREADS, 0, s>>>(n, bvec, y, r, partial, ldp, active, b.vec, sB, sP,
                                                                 b.act, sY, e);
  if (!e.ticket)
    reduce_cols_kernel<<<dim3(1, b.nsys), RED_THREADS, 0, s>>>(partial, (int)nb, ldp, 1, out, 0, active, b.res, sP,
                                                               b.act);
}

template <typename R>
void Blas<R>::scale(long long n, const R* x, R* out, const double* a, const int* active, hipStream_t s,
                    const Batch& b) const {
  constexpr int VE = 16 / sizeof(R);
  if (chunk_width<R>(n, n, b, x, out) == VE)
    scale_kernel<R, VE><<<dim3(grid_for_chunks(n / VE), 1, b.nsys), RED_THREADS, 0, s>>>(n, x, out, a, active, b.vec, b.res,
                                                                                  b.act);
  else
    scale_kernel<R, 1><<<dim3(grid_for(n), 1, b.nsys), RED_THREADS, 0, s>>>(n, x, out, a, active, b.vec, b.res,
                                                                           b.act);
}

template <typename R>
void Blas<R>::lincomb(long long n, int nsys, const R* x, long long sx, double a, const R* y, long long sy, double c,
                      R* out, long long so, const int* active, long long sA, hipStream_t s) const {
  lincomb_kernel<R><<<dim3(grid_for(n), 1, nsys), RED_THREADS, 0, s>>>(n, x, sx, a, y, sy, c, out, so, active, sA);
}

template <typename R>
void Blas<R>::fill(long long n, R* x, R v, hipStream_t s) const {
  fill_kernel<R><<<grid_for(n), RED_THREADS, 0, s>>>(n, x, v);
}

template struct Blas<double>;
template struct Blas<float>;

void cast_d2f(long long n, const double* x, float* out, const double* scale, hipStream_t s) {
  cast_scale_kernel<double, float><<<grid_for(n), RED_THREADS, 0, s>>>(n, x, out, scale, 0);
}
void axpy_f2d(long long n, const float* x, double* out, const double* scale, hipStream_t s) {
  cast_scale_kernel<float, double><<<grid_for(n), RED_THREADS, 0, s>>>(n, x, out, scale, 1);
}

}  // namespace sa

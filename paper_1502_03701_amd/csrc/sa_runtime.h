// Host-side runtime of libsa: the context and the solver drivers.
#pragma once

#include <cstdarg>
#include <map>
#include <string>
#include <vector>

#include "../../include/sa.h"
#include "blas.h"
#include "gmres_small.h"
#include "sa_internal.h"

namespace sa {

struct Buf {
  void* ptr;
  size_t bytes;
};

// An instantiated hipGraph of one GMRES restart cycle and the launch
// parameters it was captured with (buffer addresses, sizes, shifts).
struct CycleGraph {
  std::vector<unsigned char> key;
  hipGraphExec_t exec = nullptr;
};

struct Ctx {
  hipStream_t stream = nullptr;
  int device = 0;
  std::string err;
  std::map<std::string, Buf> bufs;

  bool has_base = false;
  sa_problem prob{};
  OpParams op{};
  int nv = 0;
  long long n = 0;
  double* base64 = nullptr;
  float* base32 = nullptr;
  double* bdata64 = nullptr;   // per-point base-state derivative data
  float* bdata32 = nullptr;
  // uniform thermodynamic state (op.iso points here when set)
  bool iso = false;
  IsoBase<double> iso64{};
  IsoBase<float> iso32{};

  // y = (J - shift I) x in precision R on the context's stream
  template <typename R>
  hipError_t jv(const R* x, R* y, int nrhs, double shift, const int* active) const;
  // operator kernel variant per precision ([0] FP64, [1] FP32; -1 default),
  // chosen by timing at sa_base_set unless pinned by sa_set_jv_variant
  int jv_variant[2] = {-1, -1};
  bool jv_pinned[2] = {false, false};
  float jv_tune_us[2][JV_NVARIANTS] = {};
  template <typename R>
  int variant_of() const { return jv_variant[sizeof(R) == 8 ? 0 : 1]; }

  // block-Jacobi preconditioner
  bool has_precond = false;
  int pc_nshift = 0;
  int pc_nb = 0;           // block order
  long long pc_nblocks = 0;
  int pc_bx = 0, pc_by = 0, pc_bz = 0;
  // factors, block-interleaved: [nshift][group][nb x nb entry, column-major][64 blocks]
  void* pc_lu = nullptr;   // L\U of each block
  int* pc_perm = nullptr;  // [nshift][group][nb][64] row permutation of the pivoting
  bool pc_f64 = false;     // factor precision
  int pc_kind = 0;         // SA_PC_BLOCK_JACOBI or SA_PC_MEAN_FLOW
  // mean-flow preconditioner (fourier_pc.hip): per (shift, mode) banded
  // factors, the apply's spectrum buffers and twiddle tables
  void* fp_U = nullptr;     // packed U (column length fp_ku)
  int fp_ku = 0;
  void* fp_L = nullptr;
  int* fp_piv = nullptr;
  bool fp_f64 = false;
  void *fp_specA64 = nullptr, *fp_specB64 = nullptr, *fp_specA32 = nullptr, *fp_specB32 = nullptr;
  void *fp_twx64 = nullptr, *fp_twx32 = nullptr, *fp_twz64 = nullptr, *fp_twz32 = nullptr;
  int fp_nrhs_cap = 0;

  // cached cycle graphs (captured on cap_stream, launched on stream); dropped
  // whenever the base state or the preconditioner changes
  std::vector<CycleGraph> graphs;
  hipStream_t cap_stream = nullptr;
  void drop_graphs();

  int fail(int code, const char* fmt, ...);
  int hip_fail(hipError_t e, const char* where);
  // Named, context-owned device buffer of at least `bytes` (kept across calls).
  // While `arena` is set, the buffer is carved instead from the arena (a
  // caller-independent scratch region): nothing is allocated, a name maps to
  // the same region for the rest of the call, and `zero` clears it with a
  // kernel on first use in the call.  Returns null if the arena is full.
  void* buffer(const std::string& name, size_t bytes, bool zero = true);
  struct Arena {
    unsigned char* base = nullptr;
    size_t cap = 0, used = 0;
    std::map<std::string, Buf> bufs;
  };
  Arena* arena = nullptr;
  ~Ctx();
};

// Argument checks shared by the GMRES entry points (SA_OK or the error code,
// with the message set), and their dispatch on the precision.
int gmres_check(Ctx* c, const sa_gmres_opts* o, int nshift, const double* sigma_host, const void* b_dev,
                const void* x_dev, const sa_gmres_info* info, const char* who);
int gmres_dispatch(Ctx* c, const sa_gmres_opts& o, int nshift, const double* sigma_host, const void* b_dev,
                   void* x_dev, sa_gmres_info* info);
// Device bytes the named buffers of one GMRES call take with plain launches
// (no captured cycles), each rounded up to the arena's 256-byte alignment.
size_t gmres_workspace_bytes(const Ctx* c, const sa_gmres_opts& o, int nshift);
// Zero `bytes` (rounded up to 16) at a 16-byte aligned address, by a kernel.
void zero_fill(void* p, size_t bytes, hipStream_t s);
// Resolve the device address of the allocation-free entry points' scratch
// array on the current device (once per device; sa_create calls it).
void scratch_init(int device);

template <typename R>
int solve_gmres(Ctx* c, const sa_gmres_opts& o, int nsys, const double* sigma_host, const R* b, R* x, int pc_shift0,
                sa_gmres_info* info, const std::string& tag = "g", bool io_stable = false,
                bool x0_zero = false);
// x0_zero (here and in solve_gmres): x holds zeros on entry, so the first
// residual is b (no operator product, none counted)
int solve_ir(Ctx* c, const sa_gmres_opts& o, double sigma, const double* b, double* x, int pc_shift,
             sa_gmres_info* info, bool x0_zero = false);

// mean-flow preconditioner (fourier_pc.hip): setup, and z = M^{-1} r for
// nrhs systems (at most the setup's shift count)
int fourier_setup(Ctx* c, const sa_precond_opts* o, int nshift, const double* shifts_host);
template <typename R>
hipError_t fourier_apply(Ctx* c, int ishift, int nrhs, const R* r, R* z, const int* active, int shift_step,
                         long long sV, long long sA, hipStream_t s);

// preconditioner apply z = P M^{-1} r (bjac.hip; dispatches on pc_kind)
template <typename R>
hipError_t precond_apply(Ctx* c, int ishift, int nrhs, const R* r, R* z, const int* active, int shift_step,
                         long long sV, long long sA, hipStream_t s);

}  // namespace sa

namespace sa {
template <>
inline hipError_t Ctx::jv<double>(const double* x, double* y, int nrhs, double shift, const int* active) const {
  return launch_jv<double>(op, base64, bdata64, x, y, nrhs, shift, active, stream, jv_variant[0]);
}
template <>
inline hipError_t Ctx::jv<float>(const float* x, float* y, int nrhs, double shift, const int* active) const {
  return launch_jv<float>(op, base32, bdata32, x, y, nrhs, (float)shift, active, stream, jv_variant[1]);
}
}  // namespace sa

struct sa_ctx : sa::Ctx {};

// Shared device/host definitions of the MI355X solver (gfx950, HIP).
//
// Layout conventions (all fields live in the caller's workspace):
//   node field, component q:   base + q*Nn,  Nn = N0*N1*N2, N = n + 1, x fastest
//   voxel field, comp c, ip r: base + (c*nppv + r)*Nv, Nv = n0*n1*n2
//   spectral buffers:          per component, dims change one axis per pass
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fm {

// Transform kinds of Table 1, selected by the pair of extensions at the two
// ends of an axis: P/P -> DFT, S/S -> DCT-I, A/A -> DST-I, S/A -> DCT-III,
// A/S -> DST-III.
enum Kind : int { K_DFT = 0, K_DCT1 = 1, K_DST1 = 2, K_DCT3 = 3, K_DST3 = 4 };

enum Status : int { ST_RUNNING = 0, ST_CONVERGED = 1, ST_MAXITER = 2, ST_IDLE = 3 };

// Global-memory views of pointers read from descriptors.  A pointer loaded
// from memory is generic to the compiler, which then emits flat memory
// instructions; those also count against the LDS counter, so every wait on
// one waits on the other.  Casting to the global address space gives global
// loads and stores.
#define FM_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ const FM_GLOBAL T* gconst(const T* p) { return (const FM_GLOBAL T*)p; }
template <typename T>
__device__ __forceinline__ FM_GLOBAL T* gmut(T* p) { return (FM_GLOBAL T*)p; }

constexpr int MAX_DEPTH = 4;
constexpr int MAX_RADICES = 12;
constexpr int MT_STRIDE = 160;      // reals per material table entry
constexpr int MT_VOIGT = 32;        // offset of the Voigt (engineering-shear) stiffness of an anisotropic entry
constexpr int NPART_S = 8;          // reals per stress partial: sum w|s|^2, sum s_c (6), pad
constexpr int NGRAM = 10;           // upper triangle of a 4x4 Gram matrix

// Per-solve control block (device).  Written by the control kernels, read by
// every kernel of an iteration.
struct Ctrl {
  int32_t m;              // index of the iterate being evaluated (per increment)
  int32_t status;         // Status
  int32_t aa_pending;     // Gram requested this iteration
  int32_t aa_applied;
  int32_t n_d;            // terms of the Green input  x = sum alpha_j D_{slot_d[j]}
  int32_t slot_d[MAX_DEPTH];
  int32_t n_b;            // terms of sum beta_k delta_{slot_b[k]}
  int32_t slot_b[MAX_DEPTH];
  int32_t slot_w;         // delta slot written by this iteration
  int32_t win_n;          // iterates in the history window
  int32_t win_slot[MAX_DEPTH];   // D slots of the window, oldest first
  int32_t step;
  int32_t log_count;
  int32_t max_iter, depth, period;
  int32_t mixed_mask[6];
  int32_t best_m;         // iterate of the smallest error so far (this increment)
  int32_t fp32;           // the plan stores its fields in FP32 (FM_FP32_MIXED)
  int32_t rs64;           // FP32 plan: real-space step (strain, law, divergence) now in FP64
  double alpha[MAX_DEPTH];
  double beta[MAX_DEPTH];
  double err, sumD2, sumS2;
  double best_err;        // smallest error so far (this increment)
  double macro[6];
  double c[3];
  double G[9];            // G[q*3+l]
  double H[27];           // H[(q*3+l)*3+m], symmetric in l, m
  double mixed_target[6];
  double dt, tol;
  double lam0, mu0;
  // FP32 copies read as uniform scalars by the FP32 real-space kernel:
  // G[9], H[27], tetrahedron cross terms hc[9] (h/2 H_{q,l',l''}, see k_sdiv)
  float g32[9];
  float h32[27];
  float hc32[9];
  int32_t has_trac;       // some face carries an applied traction
  // D* of the applied tractions: 2 T_q / h per [axis][face][component]
  double dstar[18];
  float dstar32[18];
};

// Refresh the FP32 copies of G, H and the TETRA2 cross terms (h_half = h/2
// for TETRA2, 0 for HEX1).
__host__ __device__ inline void ctrl_fp32_copies(Ctrl& c, double h_half) {
  for (int i = 0; i < 9; ++i) c.g32[i] = (float)c.G[i];
  for (int i = 0; i < 27; ++i) c.h32[i] = (float)c.H[i];
  for (int q = 0; q < 3; ++q) {
    c.hc32[0 * 3 + q] = (float)(h_half * c.H[(q * 3 + 1) * 3 + 2]);
    c.hc32[1 * 3 + q] = (float)(h_half * c.H[(q * 3 + 0) * 3 + 2]);
    c.hc32[2 * 3 + q] = (float)(h_half * c.H[(q * 3 + 0) * 3 + 1]);
  }
}

struct LogEntry {
  double err;
  double aa;
  double macro[6];
  uint64_t stamp;         // device wall clock at the control evaluation
  int32_t rs64;           // real-space step of this iterate evaluated in FP64
  int32_t pad_;
};

// Per-solve descriptor (device).
struct SolveDev {
  int32_t n[3], N[3];
  int64_t Nn, Nv;
  int32_t scheme, nppv, depth, has_state;
  int32_t kinds[3][3];    // [q][axis]
  double h, lam0, mu0;
  double* uf;             // 3*Nn (FP64 always)
  void* Dring;            // depth * 3 * Nn reals
  void* dring;            // depth * 3 * Nn reals
  const uint16_t* mat;    // Nv
  const void* mtab;       // material table, MT_STRIDE reals per entry
  const int32_t* mlaw;    // law per material
  void* state;            // 7 * nppv * Nv reals (or null)
  void* sig;              // plastic solves: stress of the iterate, 6 * nppv * Nv reals (or null)
  Ctrl* ctrl;
  LogEntry* log;
  double* part_s;         // ntile_s * NPART_S (stress-divergence tiles)
  double* part_d;         // ntile_d
  double* part_g;         // ntile_d * NGRAM
  int32_t ntile_s, ntile_d;
  int32_t sd_nt[3];       // stress-divergence tiles per axis (x: full-width tiles only)
  int32_t sd_zc;          // node layers per stress-divergence tile
  int32_t sd_tw;          // thread columns of the narrow x-remainder tiles
  int32_t sd_tny;         // narrow x-remainder tiles per z slab (0: none)
  int32_t wrap[3];        // axis periodic for some component
  int32_t mixed_wrap;     // some axis periodic for some components only
  double* out_u;
  double* out_eps;
  double* out_sig;
  // C0 Green operator (normal-mixed conditions only): the z pass is split
  // into a forward transform into per-component z-spectral buffers, the
  // coupled per-frequency apply, and the inverse transform
  int32_t fs;              // 1: finite-strain formulation (sig holds P^T, 9 per point)
  int32_t c0;              // 1 if the plan uses the C0 operator
  int32_t c0_cplx;         // z-spectral coefficients are complex (some axis periodic)
  int32_t c0_U[3];         // frequencies per axis, shared by the components
  int32_t c0_off[3][3];    // [q][axis]: shared frequency index - component's own index
  int32_t c0_M[3][3];      // [q][axis]: component's own extents
  int32_t c0_phase[3];     // phase of component q: (-i)^c0_phase[q]
  void* c0_spec[3];        // z-spectral buffer of component q (M0, M1, M2), x fastest
  const double* c0_sc[3];  // per axis: sin(xi/2)[U], then cos(xi/2)[U]
};

// One axis pass of one component of one solve (device).
struct PassDesc {
  int32_t solve;
  int32_t q;
  int32_t kind, n, L, nrad;
  int32_t rad[MAX_RADICES];
  int32_t cplx_in, cplx_out, packed;
  int32_t len_in, len_out;        // extent along the axis in input / output arrays
  int32_t n_p0, n_p1;             // pencil grid (p0 contiguous for strided passes)
  int32_t cols, tiles_p0;         // columns (or rows for x passes) per block
  int32_t F;                      // FFTs per block
  int64_t in_sa, in_s1, out_sa, out_s1;   // element strides
  void* in;
  void* out;
  const void* tw;                 // L twiddles exp(-2 pi i t / L)
  // x-pass extras: Anderson combination input / displacement update output
  void* ring;                     // component base of D ring (fwd) or delta ring (inv)
  int64_t ring_stride;            // reals between slots
  double* uf;                     // component base of u^f (inv x pass)
  // Green (fused z pass): per-axis tables of this component
  const double* gs2[3];           // sin^2(xi/2) per spectral index
  const double* gc2[3];           // cos^2(xi/2)
  int32_t scheme, green_lam;      // green_lam: 1 uses lambda0 (B0), 0 for 2mu0
  double h, lam0, mu0;
};

}  // namespace fm

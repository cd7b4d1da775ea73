// Host engine and C ABI of the MI355X displacement-based FFT solver.
//
// A plan carves every buffer of one solve out of the caller's workspace;
// a group (one plan, a batch, or the server's active set) owns the device
// arrays that let a single kernel launch cover the tiles of all its solves.
// The iteration loop of Algorithm 1 is nine launches; all decisions
// (convergence, Anderson schedule and weights, mixed loading) are taken on
// the device, so the host enqueues iterations in chunks and only reads a few
// status words between chunks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/fmsolve.h"
#include "fm_pass.h"
#include "fm_space.h"
#include "fm_wave.h"
#include "fm_green_c0.h"
#include "fm_finite.h"

using namespace fm;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(expr)                                                                 \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess) return fail(FM_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr size_t ALIGN = 256;
inline size_t align_up(size_t v, size_t a = ALIGN) { return (v + a - 1) / a * a; }
inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------------------
// Geometry of one solve
// ---------------------------------------------------------------------------
// Wavefront kernel for a pencil of length L: 64 lanes with E = L / 64 (E as
// in wave_E_ok), else 32 or 16 lanes per pencil with E = L / LN in {1, 3}
// (L = 16, 32, 48, 96); returns E and sets LN, or 0 when none applies.
inline int wave_shape(int L, int& LN) {
  LN = 64;
  if (L % 64 == 0 && wave_E_ok(L / 64)) return L / 64;
  for (int ln = 32; ln >= 16; ln /= 2)
    if (L % ln == 0 && (L / ln == 1 || L / ln == 3)) { LN = ln; return L / ln; }
  return 0;
}
// Tile width of the wavefront kernels: two real columns per pencil (packed)
// or one complex column, 8 wavefronts of 64 / LN pencils.
inline int wave_cols(int LN, bool packed) { return (packed ? 2 : 1) * WAVE_PENCILS * (64 / LN); }

struct Geometry {
  int n[3], N[3];
  int64_t Nn, Nv;
  int nppv, rbytes, depth;
  int kinds[3][3];
  int M[3][3];       // spectral extents [q][axis]
  int cplx[3][3];    // element complex after forward pass on axis a
  int64_t s1[3], s2[3];   // reals of stage-1 / stage-2 buffers per component
  int L[3][3];
  int F[3][7];       // FFTs per block per pass slot (generic kernel)
  int wE[3][7];      // wavefront kernel E = L / wN per pass slot, 0 = generic kernel
  int wN[3][7];      // lanes per pencil of that kernel: 64, or 32 / 16 (two / four pencils per wavefront)
  int cols[3][7];    // columns (or rows) per block per pass slot
  int c0;            // C0 Green operator: z pass split (slots 5, 6) around the coupled apply
  int64_t s3[3];     // reals of the z-spectral buffer per component (C0 only)
  int U[3];          // C0: frequencies per axis shared by the components
  int ntile_c0;      // C0: tiles of the coupled apply
  int wrap[3];       // axis periodic for some component (halo voxels take the periodic image)
  int sd_nt[3];      // fused stress-divergence tiles per axis (x: full-width tiles only)
  int sd_tw, sd_tny; // narrow x-remainder tiles: thread columns, tiles per z slab (0: none)
  int sd_zc;         // node layers per fused stress-divergence tile
  int ntile_s;       // fused stress-divergence tiles
  int ntile_v;       // voxel tiles (commit)
  int ntile_d;       // node tiles (Gram matrix)
};

int kind_of(int left, int right, int* out) {
  auto ext = [](int bc) { return bc == FM_BC_PERIODIC ? 0 : (bc == FM_BC_DIRICHLET ? -1 : 1); };
  const int a = ext(left), b = ext(right);
  if (a == 0 || b == 0) {
    if (a != b) return -1;
    *out = K_DFT;
    return 0;
  }
  if (a == 1 && b == 1) *out = K_DCT1;
  else if (a == -1 && b == -1) *out = K_DST1;
  else if (a == 1 && b == -1) *out = K_DCT3;
  else *out = K_DST3;
  return 0;
}

void factor(int L, std::vector<int>& r) {
  r.clear();
  while (L % 8 == 0 && L > 8) { r.push_back(8); L /= 8; }
  if (L == 8) { r.push_back(8); L = 1; }
  while (L % 4 == 0) { r.push_back(4); L /= 4; }
  while (L % 2 == 0) { r.push_back(2); L /= 2; }
  while (L % 3 == 0) { r.push_back(3); L /= 3; }
  while (L % 5 == 0) { r.push_back(5); L /= 5; }
  for (int p = 7; L > 1; p += 2)
    while (L % p == 0) { r.push_back(p); L /= p; }
}

// FFTs per block: bounded by the register staging of the in-place stages
// (F L <= PASS_MAXPTS) and by 16 (32 packed real columns = one 128-byte row
// segment in FP32).
int choose_F(int L, int rbytes, int cap) {
  (void)rbytes;
  int F = std::max(1, PASS_MAXPTS / std::max(L, 1));
  return std::max(1, std::min(F, cap));
}

bool generic_radix(int L) {
  std::vector<int> r;
  factor(L, r);
  for (int v : r)
    if (v != 2 && v != 3 && v != 4 && v != 5 && v != 8) return true;
  return false;
}

int make_geometry(const fm_plan_desc* d, Geometry& g) {
  if (!d) return fail(FM_E_INVALID_ARG, "null descriptor");
  for (int i = 0; i < 3; ++i) {
    if (d->n[i] < 2) return fail(FM_E_INVALID_ARG, "each grid extent must be >= 2 voxels");
    if (d->n[i] > 4096) return fail(FM_E_UNSUPPORTED, "grid extent above 4096 voxels");
    g.n[i] = d->n[i];
    g.N[i] = d->n[i] + 1;
  }
  if (!(d->h > 0)) return fail(FM_E_INVALID_ARG, "voxel size must be positive");
  if (d->scheme != FM_HEX1 && d->scheme != FM_TETRA2) return fail(FM_E_INVALID_ARG, "unknown scheme");
  if (d->green != FM_GREEN_B0 && d->green != FM_GREEN_2MU0 && d->green != FM_GREEN_C0)
    return fail(FM_E_UNSUPPORTED, "unsupported Green operator");
  if (d->prec != FM_FP64 && d->prec != FM_FP32_MIXED) return fail(FM_E_INVALID_ARG, "unknown precision");
  if (!(d->mu0 > 0) || d->lambda0 < 0) return fail(FM_E_INVALID_ARG, "reference medium needs mu0 > 0, lambda0 >= 0");
  if (d->aa_depth < 1 || d->aa_depth > MAX_DEPTH) return fail(FM_E_INVALID_ARG, "aa_depth must be in 1..4");
  if (d->aa_period < 1) return fail(FM_E_INVALID_ARG, "aa_period must be >= 1");
  if (d->max_iter < 1) return fail(FM_E_INVALID_ARG, "max_iter must be >= 1");
  if (d->max_materials < 1 || d->max_materials > 65535) return fail(FM_E_INVALID_ARG, "max_materials must be in 1..65535");
  if (d->finite_strain != 0 && d->finite_strain != 1) return fail(FM_E_INVALID_ARG, "finite_strain must be 0 or 1");
  if (d->finite_strain && d->with_state) return fail(FM_E_UNSUPPORTED, "finite-strain plans take hyperelastic laws only");
  for (int q = 0; q < 3; ++q)
    for (int i = 0; i < 3; ++i) {
      for (int a = 0; a < 2; ++a)
        if (d->bc[q][i][a] < 0 || d->bc[q][i][a] > 2) return fail(FM_E_BC, "unknown boundary condition code");
      if (kind_of(d->bc[q][i][0], d->bc[q][i][1], &g.kinds[q][i]))
        return fail(FM_E_BC, "periodic condition must hold on both opposite faces");
    }
  g.c0 = d->green == FM_GREEN_C0;
  if (g.c0) {
    // Eq. SGO_BCs: along each axis the tangential components take the
    // transform opposite to the normal one's (the periodic one stays)
    auto opposite = [](int k) {
      switch (k) { case K_DCT1: return (int)K_DST1; case K_DST1: return (int)K_DCT1; case K_DCT3: return (int)K_DST3;
                   case K_DST3: return (int)K_DCT3; default: return (int)K_DFT; }
    };
    for (int a = 0; a < 3; ++a)
      for (int q = 0; q < 3; ++q)
        if (q != a && g.kinds[q][a] != opposite(g.kinds[a][a]))
          return fail(FM_E_BC, "the C0 Green operator needs normal-mixed boundary conditions (Eq. SGO_BCs)");
  }
  g.Nn = (int64_t)g.N[0] * g.N[1] * g.N[2];
  g.Nv = (int64_t)g.n[0] * g.n[1] * g.n[2];
  g.nppv = d->scheme == FM_TETRA2 ? 2 : 1;
  g.rbytes = d->prec == FM_FP64 ? 8 : 4;
  g.depth = d->aa_depth;
  for (int q = 0; q < 3; ++q) {
    bool cx = false;
    for (int a = 0; a < 3; ++a) {
      const int k = g.kinds[q][a], n = g.n[a];
      if (k == K_DFT) { g.M[q][a] = cx ? n : n / 2 + 1; cx = true; }
      else g.M[q][a] = n_freq(k, n);
      g.cplx[q][a] = cx;
      g.L[q][a] = ext_len(k, n);
      if (g.L[q][a] > 8192) return fail(FM_E_UNSUPPORTED, "pencil too long for one LDS transform");
    }
    g.s1[q] = (int64_t)g.M[q][0] * g.N[1] * g.N[2] * (g.cplx[q][0] ? 2 : 1);
    g.s2[q] = (int64_t)g.M[q][0] * g.M[q][1] * g.N[2] * (g.cplx[q][1] ? 2 : 1);
    g.F[q][0] = choose_F(g.L[q][0], g.rbytes, 16);
    g.F[q][4] = g.F[q][0];
    g.F[q][1] = choose_F(g.L[q][1], g.rbytes, 16);
    g.F[q][3] = g.F[q][1];
    g.F[q][2] = choose_F(g.L[q][2], g.rbytes, 16);
    g.s3[q] = (int64_t)g.M[q][0] * g.M[q][1] * g.M[q][2] * (g.cplx[q][2] ? 2 : 1);
    // C0 slots 5 (z forward) and 6 (z inverse): generic kernel, strided pencils
    for (int pass = 5; pass < 7; ++pass) {
      g.F[q][pass] = g.F[q][2];
      g.wE[q][pass] = 0;
      g.wN[q][pass] = 64;
      g.cols[q][pass] = !g.cplx[q][1] ? 2 * g.F[q][pass] : g.F[q][pass];
    }
    for (int pass = 0; pass < 5; ++pass) {
      const int axis = pass == 0 || pass == 4 ? 0 : (pass == 2 ? 2 : 1);
      const int L = g.L[q][axis];
      const bool packed = axis == 0 ? true : !g.cplx[q][axis - 1];
      int LN;
      const int E = wave_shape(L, LN);
      // wavefront kernels address a component's buffers with 32-bit byte offsets
      const int64_t comp_bytes = std::max(std::max(g.s1[q], g.s2[q]) * (int64_t)g.rbytes, g.Nn * (int64_t)8);
      g.wE[q][pass] = (E && comp_bytes < ((int64_t)1 << 32)) ? E : 0;
      g.wN[q][pass] = E ? LN : 64;
      if (g.wE[q][pass]) {
        // wavefront kernel staging (bounded as in build_group) must fit the LDS
        const size_t rows = (size_t)g.n[axis] + 3;
        size_t bytes = rows * (wave_cols(LN, packed) + 1) * 2 * (size_t)g.rbytes;
        if (E == 8) bytes += (size_t)WAVE_PENCILS * WT_SIZE * g.rbytes;
        if (bytes > 150 * 1024) g.wE[q][pass] = 0;
      }
      if (g.wE[q][pass]) g.cols[q][pass] = wave_cols(LN, packed);
      else g.cols[q][pass] = packed ? 2 * g.F[q][pass] : g.F[q][pass];
      if (!g.wE[q][pass] && (generic_radix(L) ? 2 : 1) * (size_t)g.F[q][pass] * pencil_stride(L) * 2 * g.rbytes >
                                160 * 1024 - 2048)
        return fail(FM_E_UNSUPPORTED, "pencil too long for the LDS transform");
    }
  }
  for (int i = 0; i < 3; ++i) {
    g.wrap[i] = 0;
    for (int q = 0; q < 3; ++q) g.wrap[i] |= g.kinds[q][i] == K_DFT ? 1 : 0;
  }
  // 31-node x tiles; the remainder takes narrow tiles of its own width
  // (rem + 1 thread columns, SD_VT / (rem + 1) rows)
  g.sd_nt[0] = g.N[0] / SD_TX;
  g.sd_nt[1] = (int)cdiv(g.N[1], SD_TY);
  {
    const int rem = g.N[0] - g.sd_nt[0] * SD_TX;
    g.sd_tw = rem > 0 ? rem + 1 : 32;
    g.sd_tny = rem > 0 ? (int)cdiv(g.N[1], SD_VT / g.sd_tw - 1) : 0;
  }
  const int64_t sd_per_slab = (int64_t)g.sd_nt[0] * g.sd_nt[1] + g.sd_tny;
  // Layers per tile: at most SD_ZC, the node layers split evenly over the
  // z tiles; the number of z tiles doubles while the grid gives fewer than
  // 8 blocks per compute unit.  Each tile recomputes one voxel layer below
  // it, so fewer layers cost more law evaluations (elastic ones: plastic
  // solves read their stresses from the stress pass) but fill the GPU on
  // small grids; even tiles keep the last one from being a near-empty
  // block that still pays for its halo layer.
  const int64_t want = SD_WANT_BLOCKS;
  int64_t nzt = cdiv(g.N[2], SD_ZC);
  while (nzt < g.N[2] && sd_per_slab * nzt < want) nzt = std::min<int64_t>(2 * nzt, g.N[2]);
  g.sd_zc = (int)cdiv(g.N[2], nzt);
  g.sd_nt[2] = (int)cdiv(g.N[2], g.sd_zc);
  g.ntile_s = (int)(sd_per_slab * g.sd_nt[2]);
  g.ntile_v = (int)cdiv(g.Nv, SPACE_TILE);
  g.ntile_d = (int)cdiv(g.Nn, GRAM_TILE);
  g.ntile_c0 = 0;
  if (g.c0) {
    // shared frequencies per axis: the cosine transform's set for a
    // DCT-I / DST-I pair (the sine one lacks 0 and pi), else the common one
    for (int a = 0; a < 3; ++a) {
      g.U[a] = 0;
      for (int q = 0; q < 3; ++q) g.U[a] = std::max(g.U[a], g.M[q][a]);
    }
    g.ntile_c0 = (int)cdiv((int64_t)g.U[0] * g.U[1] * g.U[2], C0_TILE);
  }
  return 0;
}

// Layout of a plan workspace: offsets of every buffer.
// Blocks of one autotuning launch of a small plan's pass (its tile list
// repeated up to this count: about four per compute unit of the 256).
constexpr int FILL_BLOCKS = 1024;

struct Layout {
  size_t ctrl, log, uf, Dring, dring, specA, specB, specC, c0tab, mat, mlaw, mtab, state, sig, part_s, part_d,
      part_g, fill, tw, gtab, group, total;
  size_t tw_off[3][3];
  size_t g_off[3][3];   // green tables per comp, axis: s2 (M doubles), c2 (M doubles)
  size_t group_bytes;
};

// Work lists of a group: voxel tiles (commit), node tiles (Gram), the pass
// slots (x fwd, y fwd, fused z, y inv, x inv, and for C0 plans z fwd and
// z inv), stress-divergence tiles, C0 apply tiles.
constexpr int NPASS = 7;
constexpr int WL_VOX = 0, WL_NODE = 1, WL_PASS0 = 2, WL_SDIV = WL_PASS0 + NPASS, WL_C0 = WL_SDIV + 1;
constexpr int NWL = WL_C0 + 1;

// Pass slots a plan launches: the fused z slot for B0 / 2mu0, the split z
// slots for C0.
inline bool slot_used(const Geometry& g, int pass) {
  if (pass == 2) return !g.c0;
  if (pass >= 5) return g.c0 != 0;
  return true;
}
inline int slot_axis(int pass) { return pass == 0 || pass == 4 ? 0 : (pass == 1 || pass == 3 ? 1 : 2); }

size_t group_bytes_for(int nsolves, int64_t tiles_total[NWL]);

// Stress-divergence tiling of a group member.  A lone solve keeps the
// tiling of its geometry, which shortens the tiles until the grid fills the
// GPU; in a group whose members together give enough tiles, every member
// takes tiles of up to SD_ZC layers, since each tile recomputes one voxel
// layer below it (a one-layer tile evaluates the law twice per voxel).
// The deep tiling never has more tiles than the geometry's, for which the
// partial buffers and work lists are sized.
struct SdivTiling {
  int zc, nz, ntile;
};
inline SdivTiling sdiv_tiling(const Geometry& g, bool deep) {
  if (!deep) return {g.sd_zc, g.sd_nt[2], g.ntile_s};
  const int64_t nzt = cdiv(g.N[2], SD_ZC);
  const int zc = std::max(g.sd_zc, (int)cdiv(g.N[2], nzt));
  const int nz = (int)cdiv(g.N[2], zc);
  return {zc, nz, (g.sd_nt[0] * g.sd_nt[1] + g.sd_tny) * nz};
}

void tiles_of(const Geometry& g, int64_t t[NWL]) {
  for (int k = 0; k < NWL; ++k) t[k] = 0;
  t[WL_VOX] = g.ntile_v;
  t[WL_NODE] = g.ntile_d;
  t[WL_SDIV] = g.ntile_s;
  t[WL_C0] = g.ntile_c0;
  for (int q = 0; q < 3; ++q) {
    const int rows = g.N[1] * g.N[2];
    t[WL_PASS0 + 0] += cdiv(rows, g.cols[q][0]);
    t[WL_PASS0 + 4] += cdiv(rows, g.cols[q][4]);
    t[WL_PASS0 + 1] += cdiv(g.M[q][0], g.cols[q][1]) * g.N[2];
    t[WL_PASS0 + 3] += cdiv(g.M[q][0], g.cols[q][3]) * g.N[2];
    if (!g.c0) t[WL_PASS0 + 2] += cdiv(g.M[q][0], g.cols[q][2]) * g.M[q][1];
    else {
      t[WL_PASS0 + 5] += cdiv(g.M[q][0], g.cols[q][5]) * g.M[q][1];
      t[WL_PASS0 + 6] += cdiv(g.M[q][0], g.cols[q][6]) * g.M[q][1];
    }
  }
}

size_t group_bytes_for(int nsolves, int64_t tiles_total[NWL]) {
  size_t b = 0;
  b += align_up(sizeof(SolveDev) * nsolves);
  b += align_up(sizeof(PassDesc) * nsolves * 3 * NPASS);
  for (int i = 0; i < NWL; ++i) b += align_up(sizeof(int2) * std::max<int64_t>(1, tiles_total[i]));
  b += align_up(sizeof(int) * nsolves);
  return b;
}

void make_layout(const fm_plan_desc* d, const Geometry& g, Layout& L) {
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o += align_up(std::max<size_t>(bytes, 1)); return r; };
  const size_t R = g.rbytes;
  L.ctrl = take(sizeof(Ctrl));
  L.log = take(sizeof(LogEntry) * (size_t)(d->max_iter + 2));
  L.uf = take(8 * 3 * (size_t)g.Nn);
  L.Dring = take(R * g.depth * 3 * (size_t)g.Nn);
  L.dring = take(R * g.depth * 3 * (size_t)g.Nn);
  L.specA = take(R * (size_t)(g.s1[0] + g.s1[1] + g.s1[2]));
  L.specB = take(R * (size_t)(g.s2[0] + g.s2[1] + g.s2[2]));
  L.specC = g.c0 ? take(R * (size_t)(g.s3[0] + g.s3[1] + g.s3[2])) : 0;
  L.c0tab = g.c0 ? take(16 * (size_t)(g.U[0] + g.U[1] + g.U[2])) : 0;
  L.mat = take(2 * (size_t)g.Nv);
  L.mlaw = take(4 * (size_t)d->max_materials);
  L.mtab = take(R * MT_STRIDE * (size_t)d->max_materials);
  L.state = d->with_state ? take(R * 7 * g.nppv * (size_t)g.Nv) : 0;
  // plastic plans: sigma of the iterate (6 per point); finite strain: P^T (9 per point)
  L.sig = d->finite_strain ? take(sizeof(double) * 9 * g.nppv * (size_t)g.Nv)
          : d->with_state   ? take(R * 6 * g.nppv * (size_t)g.Nv) : 0;
  L.part_s = take(8 * NPART_S * (size_t)g.ntile_s);
  L.part_d = take(8 * (size_t)g.ntile_d);
  L.part_g = take(8 * NGRAM * (size_t)g.ntile_d);
  L.fill = take(sizeof(int2) * 5 * 2 * FILL_BLOCKS);   // repeated tile lists of the five passes (autotuner)
  for (int q = 0; q < 3; ++q)
    for (int a = 0; a < 3; ++a) L.tw_off[q][a] = take(2 * R * (size_t)g.L[q][a]);
  for (int q = 0; q < 3; ++q)
    for (int a = 0; a < 3; ++a) L.g_off[q][a] = take(16 * (size_t)g.M[q][a]);
  // sized for the most tiles any transform-kernel choice can produce (one
  // column per tile), so that fm_autotune can switch kernels in place
  Geometry gmax = g;
  for (int q = 0; q < 3; ++q)
    for (int pass = 0; pass < NPASS; ++pass) gmax.cols[q][pass] = 1;
  int64_t t[NWL];
  tiles_of(gmax, t);
  L.group_bytes = group_bytes_for(1, t);
  L.group = take(L.group_bytes);
  L.total = o + ALIGN;   // slack for base alignment
}

// ---------------------------------------------------------------------------
// Host-side material tables
// ---------------------------------------------------------------------------
void quat_rot(const double* q, double R[3][3]) {
  double w = q[0], x = q[1], y = q[2], z = q[3];
  const double nrm = std::sqrt(w * w + x * x + y * y + z * z);
  w /= nrm; x /= nrm; y /= nrm; z /= nrm;
  R[0][0] = 1 - 2 * (y * y + z * z); R[0][1] = 2 * (x * y - w * z); R[0][2] = 2 * (x * z + w * y);
  R[1][0] = 2 * (x * y + w * z); R[1][1] = 1 - 2 * (x * x + z * z); R[1][2] = 2 * (y * z - w * x);
  R[2][0] = 2 * (x * z - w * y); R[2][1] = 2 * (y * z + w * x); R[2][2] = 1 - 2 * (x * x + y * y);
}

const int MI[6] = {0, 1, 2, 1, 0, 0}, MJ[6] = {0, 1, 2, 2, 2, 1};

// Rotated cubic stiffness in Mandel form.
void cubic_mandel(double C11, double C12, double C44, const double R[3][3], double out[36]) {
  auto Cc = [&](int i, int j, int k, int l) {
    double v = C12 * (i == j) * (k == l) + C44 * ((i == k) * (j == l) + (i == l) * (j == k));
    if (i == j && j == k && k == l) v += C11 - C12 - 2 * C44;
    return v;
  };
  double Cr[3][3][3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) {
          double s = 0;
          for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
              for (int c = 0; c < 3; ++c)
                for (int e = 0; e < 3; ++e) s += R[i][a] * R[j][b] * R[k][c] * R[l][e] * Cc(a, b, c, e);
          Cr[i][j][k][l] = s;
        }
  const double w[6] = {1, 1, 1, std::sqrt(2.0), std::sqrt(2.0), std::sqrt(2.0)};
  for (int a = 0; a < 6; ++a)
    for (int b = 0; b < 6; ++b) out[a * 6 + b] = w[a] * w[b] * Cr[MI[a]][MJ[a]][MI[b]][MJ[b]];
}

// Packed upper triangle of the isotropic Voigt stiffness (lambda, mu).
void voigt_iso(double lam, double mu, double* c /* 21 */) {
  int k = 0;
  for (int i = 0; i < 6; ++i)
    for (int j = i; j < 6; ++j, ++k)
      c[k] = (i < 3 && j < 3) ? (i == j ? lam + 2 * mu : lam) : (i == j ? mu : 0.0);
}

int material_entry(const fm_material& mt, double* e /* MT_STRIDE */) {
  std::fill(e, e + MT_STRIDE, 0.0);
  switch (mt.law) {
    case FM_LAW_ISO:
      if (mt.p[0] < 0 || mt.p[1] < 0) return fail(FM_E_INVALID_ARG, "isotropic moduli must be >= 0");
      e[0] = mt.p[0]; e[1] = mt.p[1];
      voigt_iso(mt.p[0], mt.p[1], e + MT_VOIGT);
      return LAW_ISO;
    case FM_LAW_CUBIC: {
      // packed upper triangle of the (symmetric) rotated Mandel stiffness
      double R[3][3], full[36];
      quat_rot(mt.quat, R);
      cubic_mandel(mt.p[0], mt.p[1], mt.p[2], R, full);
      // and the same stiffness acting on engineering shear strains (Voigt:
      // the Mandel entries divided by sqrt(2) per shear index)
      int k = 0;
      for (int i = 0; i < 6; ++i)
        for (int j = i; j < 6; ++j) {
          const double m = 0.5 * (full[i * 6 + j] + full[j * 6 + i]);
          e[k] = m;
          e[MT_VOIGT + k] = m / ((i < 3 ? 1.0 : std::sqrt(2.0)) * (j < 3 ? 1.0 : std::sqrt(2.0)));
          ++k;
        }
      return LAW_ANISO;
    }
    case FM_LAW_J2:
      if (!(mt.p[1] > 0) || !(mt.p[2] >= 0) || !(mt.p[3] >= 0)) return fail(FM_E_INVALID_ARG, "J2 needs mu > 0, sy0 >= 0, H >= 0");
      e[0] = mt.p[0]; e[1] = mt.p[1]; e[2] = mt.p[2]; e[3] = mt.p[3];
      return LAW_J2;
    case FM_LAW_CP: {
      // the law works in the crystal frame: rotation and the three-entry
      // cubic Mandel stiffness and compliance
      const double C11 = mt.p[0], C12 = mt.p[1], C44 = mt.p[2];
      if (!(C11 > C12) || !(C11 + 2 * C12 > 0) || !(C44 > 0)) return fail(FM_E_INVALID_ARG, "singular crystal stiffness");
      double R[3][3];
      quat_rot(mt.quat, R);
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) e[i * 3 + j] = R[i][j];
      const double det = (C11 - C12) * (C11 + 2 * C12);
      e[9] = C11; e[10] = C12; e[11] = 2 * C44;
      e[12] = (C11 + C12) / det; e[13] = -C12 / det; e[14] = 1 / (2 * C44);
      if (!(mt.p[3] > 0) || !(mt.p[4] >= 1) || !(mt.p[5] > 0) || !(mt.p[6] > mt.p[5]) || !(mt.p[7] >= 0))
        return fail(FM_E_INVALID_ARG, "crystal plasticity parameters out of range");
      e[15] = mt.p[3]; e[16] = mt.p[4]; e[17] = mt.p[5]; e[18] = mt.p[6]; e[19] = mt.p[7];
      return LAW_CP;
    }
    case FM_LAW_SVK:
      if (!(mt.p[1] > 0) || !(mt.p[0] + 2.0 / 3.0 * mt.p[1] > 0)) return fail(FM_E_INVALID_ARG, "SVK needs mu > 0 and a positive bulk modulus");
      e[0] = mt.p[0]; e[1] = mt.p[1];
      return LAW_SVK;
    case FM_LAW_NEOHOOKE:
      if (!(mt.p[0] > 0) || !(mt.p[1] > 0)) return fail(FM_E_INVALID_ARG, "Neo-Hookean needs mu > 0 and K > 0");
      e[0] = mt.p[0]; e[1] = mt.p[1];
      return LAW_NEOHOOKE;
    default:
      return fail(FM_E_INVALID_ARG, "unknown law");
  }
}

__global__ void k_mat_convert(const int32_t* in, uint16_t* out, int64_t n, int nmat, int* bad) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  int v = in[i];
  if (v < 0 || v >= nmat) { atomicOr(bad, 1); v = 0; }
  out[i] = (uint16_t)v;
}

__global__ void k_cast_f(const double* in, float* out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) out[i] = (float)in[i];
}

// u^f += a v over n reals: a load step's nodal u* is folded into the
// displacement buffer for the increment (a = 1) and taken out at its end
// (a = -1), so that every kernel reads u^f + u*_nodal where it reads u^f.
// The update of an iteration adds increments that vanish on the dismissed
// nodes, so the buffer keeps the prescribed values there.
__global__ void k_add_nodal(double* __restrict__ uf, const double* __restrict__ v, double a, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) uf[i] += a * v[i];
}

__global__ void k_cast_d(const float* in, double* out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) out[i] = (double)in[i];
}

__global__ void k_copy_u16(const uint16_t* in, uint16_t* out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) out[i] = in[i];
}

}  // namespace

// ---------------------------------------------------------------------------
// Plan
// ---------------------------------------------------------------------------
struct Group;

struct fm_plan {
  fm_plan_desc d;
  Geometry g;
  Layout lay;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  SolveDev sd{};           // host image of the device descriptor
  PassDesc pd[3][NPASS]{};   // host images, per component and pass slot
  bool material_set = false;
  int n_mat = 0;
  int64_t total_iters = 0;
  Group* self = nullptr;   // single-plan group
  const double* ustar_cur = nullptr;   // nodal u* folded into u^f for the current increment
  // per-solve bookkeeping used by batch / server drivers
  int cur_step = 0;
  int rc = FM_OK;
};

// A set of solves advanced together.
// Pass kernel variants: generic (0), wavefront E = 1,2,3,4,5,6,12,16 (1-9,
// 7 unused), for E = 8 one bucket per transform kind and packing
// (10 + 2 kind + packed), whose kernels fix both at compile time, the
// 32- and 16-lane pencils with E = 1 and 3 (20-23), and per kind and packing
// (+ 2 kind + packed) the E = 3 pencils on 64 lanes (24) and on 32 lanes
// (34), and the E = 1 (44) and E = 2 (54) pencils on 64 lanes; buckets 1-3
// and 21 stay empty.
constexpr int NBUCKET = 64;
inline int bucket_of(int E, int LN, int kind, int packed) {
  const int pk = 2 * kind + (packed ? 1 : 0);
  if (E == 3 && LN >= 32) return (LN == 64 ? 24 : 34) + pk;
  if ((E == 1 || E == 2) && LN == 64) return (E == 1 ? 44 : 54) + pk;
  if (E && LN != 64) return 20 + (LN == 16 ? 2 : 0) + (E == 3 ? 1 : 0);
  switch (E) { case 1: return 1; case 2: return 2; case 3: return 3; case 4: return 4; case 5: return 5;
               case 6: return 6; case 8: return 10 + 2 * kind + (packed ? 1 : 0); case 12: return 8;
               case 16: return 9; default: return 0; }
}
constexpr int E_of_bucket[NBUCKET] = {0, 1, 2, 3, 4, 5, 6, 8, 12, 16, 8, 8, 8, 8, 8, 8, 8, 8, 8, 8, 1, 3, 1, 3,
                                      3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3, 3,
                                      1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2};

struct Group {
  int prec = 0;
  int plastic = 0;    // any solve with J2 / CP internal variables
  int trac = 0;       // some load path of the group applies tractions (real-space kernel with D*)
  bool eager = false; // launch directly, never through captured graphs
  int fs = 0;         // finite-strain solves (one formulation per group)
  int ns = 0;
  hipStream_t stream = nullptr;
  SolveDev* S = nullptr;
  PassDesc* P = nullptr;
  int2* wl[NWL]{};     // voxel, node, stress-divergence: whole lists; passes: concatenated buckets
  int64_t nwl[NWL]{};
  int64_t boff[NPASS][NBUCKET]{};   // start of each bucket inside wl[WL_PASS0 + slot]
  int64_t bn[NPASS][NBUCKET]{};     // items per bucket
  size_t blds[NPASS][NBUCKET]{};    // dynamic LDS per bucket
  int* ids = nullptr;
  // Captured iteration chunks of 1, 2, 4, ..., 32 iterations, replayed on
  // `stream`; captured on a stream of their own, dropped when the group's
  // device arrays are rebuilt.
  static constexpr int NGRAPH = 6;
  hipGraphExec_t graphs[NGRAPH] = {};
  hipStream_t cap = nullptr;
  Group() = default;
  Group(const Group&) = delete;
  Group& operator=(const Group&) = delete;
  void drop_graphs() {
    for (auto& g : graphs)
      if (g) { (void)hipGraphExecDestroy(g); g = nullptr; }
  }
  ~Group() {
    drop_graphs();
    if (cap) (void)hipStreamDestroy(cap);
  }
};

// Iteration chunks go through captured HIP graphs unless switched off
// (fm_set_graph_launch).
bool g_use_graphs = true;

bool has_traction(const fm_load_step* st, int n) {
  for (int k = 0; k < n; ++k)
    for (int i = 0; i < 18; ++i)
      if ((&st[k].traction[0][0][0])[i] != 0) return true;
  return false;
}

// Select the real-space kernel with (t) or without the traction term; the
// captured chunks hold one of them, so they are dropped on a change.
void set_trac(Group& G, bool t) {
  if (G.trac != (int)t) {
    G.drop_graphs();
    G.trac = t;
  }
}

namespace {

void fill_pass_descs(fm_plan* p) {
  const Geometry& g = p->g;
  const size_t R = g.rbytes;
  char* ws = p->ws;
  int64_t offA = 0, offB = 0, offC = 0;
  for (int q = 0; q < 3; ++q) {
    void* A = ws + p->lay.specA + R * offA;
    void* B = ws + p->lay.specB + R * offB;
    void* Cz = g.c0 ? ws + p->lay.specC + R * offC : nullptr;
    offA += g.s1[q];
    offB += g.s2[q];
    offC += g.s3[q];
    const int M2 = g.M[q][2], c3 = g.cplx[q][2];
    const int M0 = g.M[q][0], M1 = g.M[q][1];
    const int c1 = g.cplx[q][0], c2 = g.cplx[q][1];
    std::vector<int> rad;
    for (int pass = 0; pass < NPASS; ++pass) {
      PassDesc& d = p->pd[q][pass];
      std::memset(&d, 0, sizeof(d));
      d.solve = 0;
      d.q = q;
      const int axis = slot_axis(pass);
      d.kind = g.kinds[q][axis];
      d.n = g.n[axis];
      d.L = g.L[q][axis];
      factor(d.L, rad);
      d.nrad = (int)rad.size();
      for (int i = 0; i < d.nrad; ++i) d.rad[i] = rad[i];
      d.F = g.F[q][pass];
      d.tw = ws + p->lay.tw_off[q][axis];
      switch (pass) {
        case 0:   // x forward: D ring rows -> A (M0 per row)
          d.cplx_in = 0; d.cplx_out = c1; d.packed = 1;
          d.len_in = g.N[0]; d.len_out = M0;
          d.n_p0 = g.N[1] * g.N[2];
          d.cols = g.cols[q][pass];
          d.tiles_p0 = (int)cdiv(d.n_p0, d.cols);
          d.in_s1 = g.N[0]; d.out_s1 = M0;
          d.out = A;
          d.ring = ws + p->lay.Dring + R * (size_t)q * g.Nn;
          d.ring_stride = 3 * g.Nn;
          break;
        case 4:   // x inverse: A -> u update
          d.cplx_in = c1; d.cplx_out = 0; d.packed = 1;
          d.len_in = M0; d.len_out = g.N[0];
          d.n_p0 = g.N[1] * g.N[2];
          d.cols = g.cols[q][pass];
          d.tiles_p0 = (int)cdiv(d.n_p0, d.cols);
          d.in_s1 = M0; d.out_s1 = g.N[0];
          d.in = A;
          d.ring = ws + p->lay.dring + R * (size_t)q * g.Nn;
          d.ring_stride = 3 * g.Nn;
          d.uf = (double*)(ws + p->lay.uf) + (size_t)q * g.Nn;
          break;
        case 1:   // y forward: A (M0, N1, N2) -> B (M0, M1, N2)
          d.cplx_in = c1; d.cplx_out = c2; d.packed = !c1;
          d.len_in = g.N[1]; d.len_out = M1;
          d.n_p0 = M0; d.n_p1 = g.N[2];
          d.cols = g.cols[q][pass];
          d.tiles_p0 = (int)cdiv(M0, d.cols);
          d.in_sa = M0; d.in_s1 = (int64_t)M0 * g.N[1];
          d.out_sa = M0; d.out_s1 = (int64_t)M0 * M1;
          d.in = A; d.out = B;
          break;
        case 3:   // y inverse: B -> A
          d.cplx_in = c2; d.cplx_out = c1; d.packed = !c1;
          d.len_in = M1; d.len_out = g.N[1];
          d.n_p0 = M0; d.n_p1 = g.N[2];
          d.cols = g.cols[q][pass];
          d.tiles_p0 = (int)cdiv(M0, d.cols);
          d.in_sa = M0; d.in_s1 = (int64_t)M0 * M1;
          d.out_sa = M0; d.out_s1 = (int64_t)M0 * g.N[1];
          d.in = B; d.out = A;
          break;
        case 2:   // z forward + Green + inverse, in place in B (M0, M1, N2)
          d.cplx_in = c2; d.cplx_out = c2; d.packed = !c2;
          d.len_in = g.N[2]; d.len_out = g.N[2];
          d.n_p0 = M0; d.n_p1 = M1;
          d.cols = g.cols[q][pass];
          d.tiles_p0 = (int)cdiv(M0, d.cols);
          d.in_sa = d.out_sa = (int64_t)M0 * M1;
          d.in_s1 = d.out_s1 = M0;
          d.in = B; d.out = B;
          for (int a = 0; a < 3; ++a) {
            char* t = ws + p->lay.g_off[q][a];
            d.gs2[a] = (const double*)t;
            d.gc2[a] = (const double*)(t + 8 * (size_t)g.M[q][a]);
          }
          d.scheme = p->d.scheme;
          d.green_lam = p->d.green == FM_GREEN_B0;
          d.h = p->d.h; d.lam0 = p->d.lambda0; d.mu0 = p->d.mu0;
          break;
        case 5:   // C0: z forward, B (M0, M1, N2) -> C (M0, M1, M2)
          d.cplx_in = c2; d.cplx_out = c3; d.packed = !c2;
          d.len_in = g.N[2]; d.len_out = M2;
          d.n_p0 = M0; d.n_p1 = M1;
          d.cols = g.cols[q][pass];
          d.tiles_p0 = (int)cdiv(M0, d.cols);
          d.in_sa = (int64_t)M0 * M1; d.in_s1 = M0;
          d.out_sa = (int64_t)M0 * M1; d.out_s1 = M0;
          d.in = B; d.out = Cz;
          break;
        case 6:   // C0: z inverse, C -> B
          d.cplx_in = c3; d.cplx_out = c2; d.packed = !c2;
          d.len_in = M2; d.len_out = g.N[2];
          d.n_p0 = M0; d.n_p1 = M1;
          d.cols = g.cols[q][pass];
          d.tiles_p0 = (int)cdiv(M0, d.cols);
          d.in_sa = (int64_t)M0 * M1; d.in_s1 = M0;
          d.out_sa = (int64_t)M0 * M1; d.out_s1 = M0;
          d.in = Cz; d.out = B;
          break;
      }
    }
  }
}

int upload_tables(fm_plan* p) {
  const Geometry& g = p->g;
  char* ws = p->ws;
  for (int q = 0; q < 3; ++q)
    for (int a = 0; a < 3; ++a) {
      const int L = g.L[q][a];
      if (g.rbytes == 8) {
        std::vector<double> t(2 * L);
        for (int i = 0; i < L; ++i) {
          const long double ang = -2.0L * 3.14159265358979323846264338327950288L * i / L;
          t[2 * i] = (double)cosl(ang); t[2 * i + 1] = (double)sinl(ang);
        }
        HIPCHK(hipMemcpyAsync(ws + p->lay.tw_off[q][a], t.data(), 8 * t.size(), hipMemcpyHostToDevice, p->stream));
        HIPCHK(hipStreamSynchronize(p->stream));
      } else {
        std::vector<float> t(2 * L);
        for (int i = 0; i < L; ++i) {
          const long double ang = -2.0L * 3.14159265358979323846264338327950288L * i / L;
          t[2 * i] = (float)cosl(ang); t[2 * i + 1] = (float)sinl(ang);
        }
        HIPCHK(hipMemcpyAsync(ws + p->lay.tw_off[q][a], t.data(), 4 * t.size(), hipMemcpyHostToDevice, p->stream));
        HIPCHK(hipStreamSynchronize(p->stream));
      }
      // Green tables: sin^2(xi/2), cos^2(xi/2), exact 0 / 1 at the index-flagged
      // frequencies xi = 0 and xi = pi (the null-mode rule relies on it)
      const int M = g.M[q][a], n = g.n[a], k = g.kinds[q][a];
      std::vector<char> buf(16 * (size_t)M);
      double* s2 = (double*)buf.data();
      double* c2 = s2 + M;
      for (int i = 0; i < M; ++i) {
        long double xi;
        switch (k) {
          case K_DFT: xi = 2.0L * M_PIl * i / n; break;
          case K_DCT1: xi = M_PIl * i / n; break;
          case K_DST1: xi = M_PIl * (i + 1) / n; break;
          default: xi = M_PIl * (i + 0.5L) / n; break;
        }
        uint8_t f = 0;
        if ((k == K_DFT || k == K_DCT1) && i == 0) f |= 1;
        if ((k == K_DFT && n % 2 == 0 && i == n / 2) || (k == K_DCT1 && i == n)) f |= 2;
        long double s = sinl(0.5L * xi), c = cosl(0.5L * xi);
        if (f & 1) { s = 0; c = 1; }
        if (f & 2) { s = 1; c = 0; }
        s2[i] = (double)(s * s);
        c2[i] = (double)(c * c);
      }
      HIPCHK(hipMemcpyAsync(ws + p->lay.g_off[q][a], buf.data(), buf.size(), hipMemcpyHostToDevice, p->stream));
      HIPCHK(hipStreamSynchronize(p->stream));
    }
  if (g.c0) {
    // C0: sin(xi/2) and cos(xi/2) (signed: a full periodic axis reaches
    // xi > pi) of each shared frequency per axis, exact 0 / 1 at xi = 0, pi
    std::vector<double> t;
    for (int a = 0; a < 3; ++a) {
      const int n = g.n[a], U = g.U[a];
      const int kn = g.kinds[a][a];   // the normal component's transform fixes the frequency set
      std::vector<double> sv(U), cv(U);
      for (int u = 0; u < U; ++u) {
        long double xi;
        bool z = false, pi = false;
        if (kn == K_DFT) { xi = 2.0L * M_PIl * u / n; z = u == 0; pi = 2 * u == n; }
        else if (kn == K_DCT1 || kn == K_DST1) { xi = M_PIl * u / n; z = u == 0; pi = u == n; }
        else xi = M_PIl * (u + 0.5L) / n;
        sv[u] = z ? 0.0 : pi ? 1.0 : (double)sinl(0.5L * xi);
        cv[u] = z ? 1.0 : pi ? 0.0 : (double)cosl(0.5L * xi);
      }
      t.insert(t.end(), sv.begin(), sv.end());
      t.insert(t.end(), cv.begin(), cv.end());
    }
    HIPCHK(hipMemcpyAsync(ws + p->lay.c0tab, t.data(), 8 * t.size(), hipMemcpyHostToDevice, p->stream));
    HIPCHK(hipStreamSynchronize(p->stream));
  }
  return 0;
}

// Workgroups are dealt to the XCDs round robin (block b to XCD b mod 8).
// Reorder a work list segment so that each XCD receives a contiguous run of
// the spatial order: neighbouring tiles then share halos and partial cache
// lines through the same L2.
constexpr int N_XCD = 8;
void xcd_order(std::vector<int2>& v, size_t begin, size_t end) {
  const size_t T = end - begin;
  if (T < 2 * N_XCD) return;
  std::vector<int2> out(T);
  size_t start[N_XCD];
  size_t acc = 0;
  for (int k = 0; k < N_XCD; ++k) {
    start[k] = acc;
    acc += T / N_XCD + ((size_t)k < T % N_XCD ? 1 : 0);
  }
  for (size_t b = 0; b < T; ++b) out[b] = v[begin + start[b % N_XCD] + b / N_XCD];
  std::copy(out.begin(), out.end(), v.begin() + begin);
}

// Build a group's device arrays for `plans` inside [dev, dev+bytes).
int build_group(Group& G, fm_plan* const* plans, int ns, char* dev, size_t bytes, hipStream_t stream) {
  if (ns < 1) return fail(FM_E_INVALID_ARG, "empty group");
  G.drop_graphs();
  G.prec = plans[0]->d.prec;
  G.ns = ns;
  G.plastic = 0;
  for (int i = 0; i < ns; ++i) G.plastic |= plans[i]->d.with_state ? 1 : 0;
  G.fs = plans[0]->d.finite_strain;
  for (int i = 0; i < ns; ++i)
    if (plans[i]->d.finite_strain != G.fs) return fail(FM_E_INVALID_ARG, "a batch must share one formulation (small or finite strain)");
  G.stream = stream;
  int64_t t[NWL] = {};
  for (int i = 0; i < ns; ++i) {
    if (plans[i]->d.prec != G.prec) return fail(FM_E_INVALID_ARG, "a batch must share one precision");
    int64_t ti[NWL];
    tiles_of(plans[i]->g, ti);
    for (int k = 0; k < NWL; ++k) t[k] += ti[k];
  }
  const size_t need = group_bytes_for(ns, t);
  if (need > bytes) return fail(FM_E_WORKSPACE, "group workspace too small");
  size_t o = 0;
  G.S = (SolveDev*)(dev + o); o += align_up(sizeof(SolveDev) * ns);
  G.P = (PassDesc*)(dev + o); o += align_up(sizeof(PassDesc) * ns * 3 * NPASS);
  for (int k = 0; k < NWL; ++k) { G.wl[k] = (int2*)(dev + o); o += align_up(sizeof(int2) * std::max<int64_t>(1, t[k])); }
  G.ids = (int*)(dev + o);
  std::vector<SolveDev> S(ns);
  std::vector<PassDesc> P((size_t)ns * 3 * NPASS);
  std::vector<int2> wl[4];          // voxel, node, stress-divergence, C0 apply tiles
  std::vector<int2> pb[NPASS][NBUCKET];
  std::vector<int> ids(ns);
  for (int k = 0; k < NPASS; ++k)
    for (int b = 0; b < NBUCKET; ++b) G.blds[k][b] = 0;
  int64_t deep_tiles = 0;
  for (int i = 0; i < ns; ++i) deep_tiles += sdiv_tiling(plans[i]->g, true).ntile;
  const bool deep = ns > 1 && deep_tiles >= SD_WANT_BLOCKS;
  for (int i = 0; i < ns; ++i) {
    fm_plan* p = plans[i];
    S[i] = p->sd;
    const SdivTiling st = sdiv_tiling(p->g, deep);
    S[i].sd_zc = st.zc;
    S[i].sd_nt[2] = st.nz;
    S[i].ntile_s = st.ntile;
    ids[i] = i;
    for (int ty = 0; ty < p->g.ntile_v; ++ty) wl[0].push_back(make_int2(i, ty));
    for (int ty = 0; ty < p->g.ntile_d; ++ty) wl[1].push_back(make_int2(i, ty));
    for (int ty = 0; ty < st.ntile; ++ty) wl[2].push_back(make_int2(i, ty));
    for (int ty = 0; ty < p->g.ntile_c0; ++ty) wl[3].push_back(make_int2(i, ty));
    for (int q = 0; q < 3; ++q)
      for (int pass = 0; pass < NPASS; ++pass) {
        PassDesc d = p->pd[q][pass];
        d.solve = i;
        const int di = (i * 3 + q) * NPASS + pass;
        P[di] = d;
        if (!slot_used(p->g, pass)) continue;
        const int64_t ntiles = pass == 0 || pass == 4 ? d.tiles_p0 : (int64_t)d.tiles_p0 * d.n_p1;
        const int pk = pass;   // launch order slot
        const int E = p->g.wE[q][pass], LN = p->g.wN[q][pass];
        const int b = bucket_of(E, LN, d.kind, d.packed);
        if (E && (d.cols != wave_cols(LN, d.packed) || d.L != LN * E))
          return fail(FM_E_INVALID_ARG, "internal: wavefront pass descriptor does not match its kernel");
        for (int64_t ty = 0; ty < ntiles; ++ty) pb[pk][b].push_back(make_int2(di, (int)ty));
        size_t lds;
        const size_t R = p->g.rbytes;
        if (E) {
          // staging of phase A (input tile) and phase C (output tile), sized separately
          const int mode = pass == 2 ? 2 : (pass == 3 || pass == 4 || pass == 6) ? 1 : 0;
          const bool half = d.packed && d.kind == K_DFT;
          int j0, cnt;
          raw_range(d.kind, d.n, j0, cnt);
          const int rows_in = mode == 1 ? d.len_in : cnt;
          const size_t es_in = d.cplx_in ? 2 * R : R;
          const int M = half ? d.n / 2 + 1 : n_freq(d.kind, d.n);
          const int rows_out = mode == 0 ? M : d.n + 1;
          const size_t es_out = mode == 0 ? (d.cplx_out ? 2 * R : R) : (d.packed ? R : 2 * R);
          lds = std::max((size_t)(rows_in + 2) * (d.cols + 1) * es_in, (size_t)(rows_out + 2) * (d.cols + 1) * es_out);
          if (E == 8) lds += (size_t)WAVE_PENCILS * WT_SIZE * R;   // transpose scratch
        } else {
          lds = (generic_radix(d.L) ? 2 : 1) * (size_t)d.F * pencil_stride(d.L) * 2 * R;
        }
        G.blds[pk][b] = std::max(G.blds[pk][b], lds);
      }
  }
  std::vector<int2> pl[NPASS];
  for (int k = 0; k < NPASS; ++k) {
    int64_t off = 0;
    for (int b = 0; b < NBUCKET; ++b) {
      G.boff[k][b] = off;
      G.bn[k][b] = (int64_t)pb[k][b].size();
      pl[k].insert(pl[k].end(), pb[k][b].begin(), pb[k][b].end());
      xcd_order(pl[k], (size_t)off, (size_t)(off + G.bn[k][b]));
      off += G.bn[k][b];
    }
  }
  for (int k = 0; k < 4; ++k) xcd_order(wl[k], 0, wl[k].size());
  HIPCHK(hipMemcpyAsync(G.S, S.data(), sizeof(SolveDev) * ns, hipMemcpyHostToDevice, stream));
  HIPCHK(hipMemcpyAsync(G.P, P.data(), sizeof(PassDesc) * P.size(), hipMemcpyHostToDevice, stream));
  for (int k = 0; k < NWL; ++k) {
    const std::vector<int2>& v = k == WL_VOX ? wl[0] : k == WL_NODE ? wl[1] : k == WL_SDIV ? wl[2]
                                 : k == WL_C0 ? wl[3] : pl[k - WL_PASS0];
    G.nwl[k] = (int64_t)v.size();
    if (!v.empty())
      HIPCHK(hipMemcpyAsync(G.wl[k], v.data(), sizeof(int2) * v.size(), hipMemcpyHostToDevice, stream));
  }
  HIPCHK(hipMemcpyAsync(G.ids, ids.data(), sizeof(int) * ns, hipMemcpyHostToDevice, stream));
  HIPCHK(hipStreamSynchronize(stream));
  return 0;
}

// Persistent pipelined form of the strided E = 8 passes (FP32): at most
// P_BLOCKS_PER_CU blocks per compute unit, a multiple of 8 blocks in all.
constexpr int P_BLOCKS_PER_CU = 4;
int g_num_cu = 0;

// Resident blocks per compute unit of a kernel at a given dynamic LDS size
// (cached: the launch path is also captured into graphs).
inline int resident_blocks(const void* f, size_t lds) {
  static std::map<std::pair<const void*, size_t>, int> cache;
  static std::mutex mu;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find({f, lds});
  if (it != cache.end()) return it->second;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, WAVE_THREADS, lds) != hipSuccess) nb = 1;
  nb = std::max(1, std::min(nb, P_BLOCKS_PER_CU));
  cache[{f, lds}] = nb;
  return nb;
}

template <int MODE, int KIND>
void launch_w8p(int packed, int nwork, size_t lds, hipStream_t st, const PassDesc* P, const int2* wl,
                const SolveDev* S) {
  lds += p_extra_lds(MODE, KIND, packed);
  const void* f = packed ? (const void*)k_wave_p<MODE, KIND, 1> : (const void*)k_wave_p<MODE, KIND, 0>;
  int G = std::min(nwork, resident_blocks(f, lds) * g_num_cu);
  if (G >= 8) G -= G % 8;
  if (packed) hipLaunchKernelGGL((k_wave_p<MODE, KIND, 1>), dim3(G), dim3(WAVE_THREADS), lds, st, P, wl, nwork, S);
  else hipLaunchKernelGGL((k_wave_p<MODE, KIND, 0>), dim3(G), dim3(WAVE_THREADS), lds, st, P, wl, nwork, S);
}

template <int MODE>
void launch_w8p_kind(int kind, int packed, int nwork, size_t lds, hipStream_t st, const PassDesc* P,
                     const int2* wl, const SolveDev* S) {
  switch (kind) {
    case K_DFT: launch_w8p<MODE, K_DFT>(packed, nwork, lds, st, P, wl, S); break;
    case K_DCT1: launch_w8p<MODE, K_DCT1>(packed, nwork, lds, st, P, wl, S); break;
    case K_DST1: launch_w8p<MODE, K_DST1>(packed, nwork, lds, st, P, wl, S); break;
    case K_DCT3: launch_w8p<MODE, K_DCT3>(packed, nwork, lds, st, P, wl, S); break;
    default: launch_w8p<MODE, K_DST3>(packed, nwork, lds, st, P, wl, S); break;
  }
}

template <int MODE, int KIND>
void launch_w8px(int nwork, size_t lds, hipStream_t st, const PassDesc* P, const int2* wl, const SolveDev* S) {
  lds += px_extra_lds();
  const void* f = (const void*)k_wave_px<MODE, KIND>;
  int G = std::min(nwork, resident_blocks(f, lds) * g_num_cu);
  if (G >= 8) G -= G % 8;
  hipLaunchKernelGGL((k_wave_px<MODE, KIND>), dim3(G), dim3(WAVE_THREADS), lds, st, P, wl, nwork, S);
}

template <int MODE>
void launch_w8px_kind(int kind, int nwork, size_t lds, hipStream_t st, const PassDesc* P, const int2* wl,
                      const SolveDev* S) {
  switch (kind) {
    case K_DFT: launch_w8px<MODE, K_DFT>(nwork, lds, st, P, wl, S); break;
    case K_DCT1: launch_w8px<MODE, K_DCT1>(nwork, lds, st, P, wl, S); break;
    case K_DST1: launch_w8px<MODE, K_DST1>(nwork, lds, st, P, wl, S); break;
    case K_DCT3: launch_w8px<MODE, K_DCT3>(nwork, lds, st, P, wl, S); break;
    default: launch_w8px<MODE, K_DST3>(nwork, lds, st, P, wl, S); break;
  }
}

template <int MODE>
hipError_t set_w8px_lds_kinds(int big) {
  hipError_t r;
  if ((r = hipFuncSetAttribute((const void*)k_wave_px<MODE, K_DFT>, hipFuncAttributeMaxDynamicSharedMemorySize, big))) return r;
  if ((r = hipFuncSetAttribute((const void*)k_wave_px<MODE, K_DCT1>, hipFuncAttributeMaxDynamicSharedMemorySize, big))) return r;
  if ((r = hipFuncSetAttribute((const void*)k_wave_px<MODE, K_DST1>, hipFuncAttributeMaxDynamicSharedMemorySize, big))) return r;
  if ((r = hipFuncSetAttribute((const void*)k_wave_px<MODE, K_DCT3>, hipFuncAttributeMaxDynamicSharedMemorySize, big))) return r;
  return hipFuncSetAttribute((const void*)k_wave_px<MODE, K_DST3>, hipFuncAttributeMaxDynamicSharedMemorySize, big);
}

template <int MODE, int KIND>
hipError_t set_w8p_lds(int big) {
  hipError_t r = hipFuncSetAttribute((const void*)k_wave_p<MODE, KIND, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, big);
  if (r) return r;
  return hipFuncSetAttribute((const void*)k_wave_p<MODE, KIND, 0>, hipFuncAttributeMaxDynamicSharedMemorySize, big);
}

template <int MODE>
hipError_t set_w8p_lds_kinds(int big) {
  hipError_t r;
  if ((r = set_w8p_lds<MODE, K_DFT>(big))) return r;
  if ((r = set_w8p_lds<MODE, K_DCT1>(big))) return r;
  if ((r = set_w8p_lds<MODE, K_DST1>(big))) return r;
  if ((r = set_w8p_lds<MODE, K_DCT3>(big))) return r;
  return set_w8p_lds<MODE, K_DST3>(big);
}

template <typename R, int MODE, int XP, int KIND>
hipError_t set_w8_lds(int big) {
  hipError_t r = hipFuncSetAttribute((const void*)k_wave<R, MODE, XP, 8, KIND, 1>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, big);
  if (r) return r;
  if constexpr (!XP)
    r = hipFuncSetAttribute((const void*)k_wave<R, MODE, XP, 8, KIND, 0>, hipFuncAttributeMaxDynamicSharedMemorySize, big);
  return r;
}

template <typename R, int MODE, int XP>
hipError_t set_w8_lds_kinds(int big) {
  hipError_t r;
  if ((r = set_w8_lds<R, MODE, XP, K_DFT>(big))) return r;
  if ((r = set_w8_lds<R, MODE, XP, K_DCT1>(big))) return r;
  if ((r = set_w8_lds<R, MODE, XP, K_DST1>(big))) return r;
  if ((r = set_w8_lds<R, MODE, XP, K_DCT3>(big))) return r;
  return set_w8_lds<R, MODE, XP, K_DST3>(big);
}

template <typename R, int E>
hipError_t set_wave_lds(int big) {
  if constexpr (E == 8) {
    hipError_t r;
    if ((r = set_w8_lds_kinds<R, 0, 1>(big))) return r;
    if ((r = set_w8_lds_kinds<R, 1, 1>(big))) return r;
    if ((r = set_w8_lds_kinds<R, 0, 0>(big))) return r;
    if ((r = set_w8_lds_kinds<R, 1, 0>(big))) return r;
    return set_w8_lds_kinds<R, 2, 0>(big);
  } else {
    hipError_t r;
    if ((r = hipFuncSetAttribute((const void*)k_wave<R, 0, 1, E>, hipFuncAttributeMaxDynamicSharedMemorySize, big))) return r;
    if ((r = hipFuncSetAttribute((const void*)k_wave<R, 1, 1, E>, hipFuncAttributeMaxDynamicSharedMemorySize, big))) return r;
    if ((r = hipFuncSetAttribute((const void*)k_wave<R, 0, 0, E>, hipFuncAttributeMaxDynamicSharedMemorySize, big))) return r;
    if ((r = hipFuncSetAttribute((const void*)k_wave<R, 1, 0, E>, hipFuncAttributeMaxDynamicSharedMemorySize, big))) return r;
    return hipFuncSetAttribute((const void*)k_wave<R, 2, 0, E>, hipFuncAttributeMaxDynamicSharedMemorySize, big);
  }
}

template <typename R, int TR>
hipError_t set_sdiv_lds_tr() {
  hipError_t r;
  if ((r = hipFuncSetAttribute((const void*)k_sdiv<R, 0, R, TR>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)sdiv_lds_bytes(sizeof(R)))))
    return r;
  if ((r = hipFuncSetAttribute((const void*)k_sdiv<R, 1, R, TR>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)sdiv_lds_bytes(sizeof(R)))))
    return r;
  if constexpr (sizeof(R) == 4) {
    if ((r = hipFuncSetAttribute((const void*)k_sdiv<R, 0, double, TR>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)sdiv_lds_bytes(8))))
      return r;
    return hipFuncSetAttribute((const void*)k_sdiv<R, 1, double, TR>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)sdiv_lds_bytes(8));
  }
  return hipSuccess;
}

template <typename R>
hipError_t set_sdiv_lds() {
  hipError_t r = set_sdiv_lds_tr<R, 0>();
  if (r) return r;
  return set_sdiv_lds_tr<R, 1>();
}

template <typename R>
int set_lds_limits() {
  static bool done = false;
  if (done) return 0;
  const int big = 160 * 1024 - 2048;   // leave room for static shared arrays
  HIPCHK(hipFuncSetAttribute((const void*)k_pass<R, 0, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, big));
  HIPCHK(hipFuncSetAttribute((const void*)k_pass<R, 1, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, big));
  HIPCHK(hipFuncSetAttribute((const void*)k_pass<R, 0, 0>, hipFuncAttributeMaxDynamicSharedMemorySize, big));
  HIPCHK(hipFuncSetAttribute((const void*)k_pass<R, 1, 0>, hipFuncAttributeMaxDynamicSharedMemorySize, big));
  HIPCHK(hipFuncSetAttribute((const void*)k_pass<R, 2, 0>, hipFuncAttributeMaxDynamicSharedMemorySize, big));
  HIPCHK((set_wave_lds<R, 1>(big)));
  HIPCHK((set_wave_lds<R, 2>(big)));
  HIPCHK((set_wave_lds<R, 3>(big)));
  HIPCHK((set_wave_lds<R, 4>(big)));
  HIPCHK((set_wave_lds<R, 5>(big)));
  HIPCHK((set_wave_lds<R, 6>(big)));
  HIPCHK((set_wave_lds<R, 8>(big)));
  if constexpr (sizeof(R) == 4) {
    HIPCHK(set_w8p_lds_kinds<0>(big));
    HIPCHK(set_w8p_lds_kinds<1>(big));
    HIPCHK(set_w8p_lds_kinds<2>(big));
    HIPCHK(set_w8px_lds_kinds<0>(big));
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&g_num_cu, hipDeviceAttributeMultiprocessorCount, dev));
  }
  HIPCHK((set_wave_lds<R, 12>(big)));
  HIPCHK((set_wave_lds<R, 16>(big)));
  HIPCHK(set_sdiv_lds<R>());
  done = true;
  return 0;
}

// E = 8 kernels specialised on kind and packing (x passes are always packed;
// the fused z pass only runs strided).
template <typename R, int MODE, int XP, int KIND>
void launch_w8(int packed, dim3 grid, size_t lds, hipStream_t st, const PassDesc* P, const int2* wl,
               const SolveDev* S) {
  if (packed) hipLaunchKernelGGL((k_wave<R, MODE, XP, 8, KIND, 1>), grid, dim3(WAVE_THREADS), lds, st, P, wl, S);
  else if constexpr (!XP) hipLaunchKernelGGL((k_wave<R, MODE, XP, 8, KIND, 0>), grid, dim3(WAVE_THREADS), lds, st, P, wl, S);
}

template <typename R, int MODE, int XP>
void launch_w8_kind(int kind, int packed, dim3 grid, size_t lds, hipStream_t st, const PassDesc* P,
                    const int2* wl, const SolveDev* S) {
  if constexpr (!XP && sizeof(R) == 4) {
    if (g_num_cu > 0) {
      launch_w8p_kind<MODE>(kind, packed, (int)grid.x, lds, st, P, wl, S);
      return;
    }
  } else if constexpr (XP && MODE == 0 && sizeof(R) == 4) {
    // (the x inverse pass stays one tile per block: its u^f update reads
    // global memory after the transform, and those waits would take in the
    // prefetch; measured slower pipelined)
    if (g_num_cu > 0 && packed) {
      launch_w8px_kind<MODE>(kind, (int)grid.x, lds, st, P, wl, S);
      return;
    }
  }
  switch (kind) {
    case K_DFT: launch_w8<R, MODE, XP, K_DFT>(packed, grid, lds, st, P, wl, S); break;
    case K_DCT1: launch_w8<R, MODE, XP, K_DCT1>(packed, grid, lds, st, P, wl, S); break;
    case K_DST1: launch_w8<R, MODE, XP, K_DST1>(packed, grid, lds, st, P, wl, S); break;
    case K_DCT3: launch_w8<R, MODE, XP, K_DCT3>(packed, grid, lds, st, P, wl, S); break;
    default: launch_w8<R, MODE, XP, K_DST3>(packed, grid, lds, st, P, wl, S); break;
  }
}

// The pencils of grids of 32-96 cells (L = 64, 128 and 192 on 64 lanes, L =
// 96 on 32): in FP32 compiled per transform kind and packing like the E = 8
// kernels (n, element types and pitches fixed at compile time), in FP64 the
// descriptor-driven kernel.  Returns false for a combination that has no
// kernel (x passes are always packed).
template <int MODE, int XP, int E, int LN, int KIND>
bool launch_wks(int packed, dim3 grid, size_t lds, hipStream_t st, const PassDesc* P, const int2* wl,
                const SolveDev* S) {
  if (packed) {
    hipLaunchKernelGGL((k_wave<float, MODE, XP, E, KIND, 1, LN>), grid, dim3(WAVE_THREADS), lds, st, P, wl, S);
    return true;
  }
  if constexpr (!XP) {
    hipLaunchKernelGGL((k_wave<float, MODE, XP, E, KIND, 0, LN>), grid, dim3(WAVE_THREADS), lds, st, P, wl, S);
    return true;
  }
  return false;
}

template <typename R, int MODE, int XP, int E, int LN>
bool launch_wk(int kind, int packed, dim3 grid, size_t lds, hipStream_t st, const PassDesc* P, const int2* wl,
               const SolveDev* S) {
  if constexpr (sizeof(R) == 4) {
    switch (kind) {
      case K_DFT: return launch_wks<MODE, XP, E, LN, K_DFT>(packed, grid, lds, st, P, wl, S);
      case K_DCT1: return launch_wks<MODE, XP, E, LN, K_DCT1>(packed, grid, lds, st, P, wl, S);
      case K_DST1: return launch_wks<MODE, XP, E, LN, K_DST1>(packed, grid, lds, st, P, wl, S);
      case K_DCT3: return launch_wks<MODE, XP, E, LN, K_DCT3>(packed, grid, lds, st, P, wl, S);
      default: return launch_wks<MODE, XP, E, LN, K_DST3>(packed, grid, lds, st, P, wl, S);
    }
  } else {
    hipLaunchKernelGGL((k_wave<R, MODE, XP, E, -1, -1, LN>), grid, dim3(WAVE_THREADS), lds, st, P, wl, S);
    return true;
  }
}

template <typename R, int MODE, int XP>
int launch_bucket(const Group& G, int pk, int b) {
  const int2* wl = G.wl[WL_PASS0 + pk] + G.boff[pk][b];
  const dim3 grid((unsigned)G.bn[pk][b]);
  const size_t lds = G.blds[pk][b];
  hipStream_t st = G.stream;
  if (b >= 24) {
    const int set = (b - 24) / 10, kind = ((b - 24) % 10) >> 1, packed = b & 1;
    bool ok;
    switch (set) {
      case 0: ok = launch_wk<R, MODE, XP, 3, 64>(kind, packed, grid, lds, st, G.P, wl, G.S); break;
      case 1: ok = launch_wk<R, MODE, XP, 3, 32>(kind, packed, grid, lds, st, G.P, wl, G.S); break;
      case 2: ok = launch_wk<R, MODE, XP, 1, 64>(kind, packed, grid, lds, st, G.P, wl, G.S); break;
      default: ok = launch_wk<R, MODE, XP, 2, 64>(kind, packed, grid, lds, st, G.P, wl, G.S); break;
    }
    if (!ok) return fail(FM_E_INVALID_ARG, "internal: no wavefront kernel for an unpacked x pass");
  } else if (b >= 20) {
    switch (b) {
      case 20: hipLaunchKernelGGL((k_wave<R, MODE, XP, 1, -1, -1, 32>), grid, dim3(WAVE_THREADS), lds, st, G.P, wl, G.S); break;
      case 21: hipLaunchKernelGGL((k_wave<R, MODE, XP, 3, -1, -1, 32>), grid, dim3(WAVE_THREADS), lds, st, G.P, wl, G.S); break;
      case 22: hipLaunchKernelGGL((k_wave<R, MODE, XP, 1, -1, -1, 16>), grid, dim3(WAVE_THREADS), lds, st, G.P, wl, G.S); break;
      default: hipLaunchKernelGGL((k_wave<R, MODE, XP, 3, -1, -1, 16>), grid, dim3(WAVE_THREADS), lds, st, G.P, wl, G.S); break;
    }
  } else if (b >= 10) {
    launch_w8_kind<R, MODE, XP>((b - 10) >> 1, (b - 10) & 1, grid, lds, st, G.P, wl, G.S);
  } else switch (E_of_bucket[b]) {
    case 0: hipLaunchKernelGGL((k_pass<R, MODE, XP>), grid, dim3(PASS_THREADS), lds, st, G.P, wl, G.S); break;
    case 1: hipLaunchKernelGGL((k_wave<R, MODE, XP, 1>), grid, dim3(WAVE_THREADS), lds, st, G.P, wl, G.S); break;
    case 2: hipLaunchKernelGGL((k_wave<R, MODE, XP, 2>), grid, dim3(WAVE_THREADS), lds, st, G.P, wl, G.S); break;
    case 3: hipLaunchKernelGGL((k_wave<R, MODE, XP, 3>), grid, dim3(WAVE_THREADS), lds, st, G.P, wl, G.S); break;
    case 4: hipLaunchKernelGGL((k_wave<R, MODE, XP, 4>), grid, dim3(WAVE_THREADS), lds, st, G.P, wl, G.S); break;
    case 5: hipLaunchKernelGGL((k_wave<R, MODE, XP, 5>), grid, dim3(WAVE_THREADS), lds, st, G.P, wl, G.S); break;
    case 6: hipLaunchKernelGGL((k_wave<R, MODE, XP, 6>), grid, dim3(WAVE_THREADS), lds, st, G.P, wl, G.S); break;
    case 12: hipLaunchKernelGGL((k_wave<R, MODE, XP, 12>), grid, dim3(WAVE_THREADS), lds, st, G.P, wl, G.S); break;
    default: hipLaunchKernelGGL((k_wave<R, MODE, XP, 16>), grid, dim3(WAVE_THREADS), lds, st, G.P, wl, G.S); break;
  }
  const hipError_t err = hipGetLastError();
  if (err != hipSuccess)
    return fail(FM_E_HIP, std::string("pass launch (mode ") + std::to_string(MODE) + ", x " + std::to_string(XP) +
                              ", E " + std::to_string(E_of_bucket[b]) + ", lds " + std::to_string(lds) +
                              ", grid " + std::to_string(G.bn[pk][b]) + "): " + hipGetErrorString(err));
  return 0;
}

template <typename R>
int launch_pass(const Group& G, int pk, int b) {
  switch (pk) {
    case 0: return launch_bucket<R, 0, 1>(G, pk, b);
    case 1: return launch_bucket<R, 0, 0>(G, pk, b);
    case 2: return launch_bucket<R, 2, 0>(G, pk, b);
    case 3: return launch_bucket<R, 1, 0>(G, pk, b);
    case 5: return launch_bucket<R, 0, 0>(G, pk, b);
    case 6: return launch_bucket<R, 1, 0>(G, pk, b);
    default: return launch_bucket<R, 1, 1>(G, pk, b);
  }
}

template <typename R>
int launch_slot(const Group& G, int pk) {
  for (int b = 0; b < NBUCKET; ++b)
    if (G.bn[pk][b]) {
      const int rc = launch_pass<R>(G, pk, b);
      if (rc) return rc;
    }
  return 0;
}

// Blocks of the FP64 real-space kernel of FP32 groups: two per compute unit,
// walking the tile list (a multiple of 8, so each stays on one XCD).
inline int rs64_grid(const Group& G) {
  const int cu = g_num_cu > 0 ? g_num_cu : 256;
  return (int)std::max<int64_t>(1, std::min<int64_t>(G.nwl[WL_SDIV], 2 * cu));
}

template <typename R, int TR>
int launch_sdiv(const Group& G) {
  hipStream_t st = G.stream;
  const int nw = (int)G.nwl[WL_SDIV];
  if (G.fs) {
    // finite strain: P per voxel (FP64 law, R storage), then its divergence
    if (G.nwl[WL_VOX])
      hipLaunchKernelGGL((k_fs_stress<R>), dim3(G.nwl[WL_VOX] * (SPACE_TILE / 256)), dim3(256), 0, st, G.S,
                         G.wl[WL_VOX]);
    hipLaunchKernelGGL((k_fs_div<R>), dim3(nw), dim3(256), 0, st, G.S, G.wl[WL_SDIV]);
    HIPCHK(hipGetLastError());
    return 0;
  }
  // FP32 groups launch the FP32 and the FP64 real-space kernel; each solve's
  // control block picks the one that works (the other returns)
  if (G.plastic) {
    // plastic solves: the law once per voxel (one thread each), then the
    // fused kernel reads those stresses
    if (G.nwl[WL_VOX])
      hipLaunchKernelGGL((k_commit<R, 1, 1>), dim3(G.nwl[WL_VOX] * (SPACE_TILE / 256)), dim3(256), 0, st, G.S,
                         G.wl[WL_VOX]);
    hipLaunchKernelGGL((k_sdiv<R, 1, R, TR>), dim3(nw), dim3(256), sdiv_lds_bytes(sizeof(R)), st, G.S, G.wl[WL_SDIV], nw);
    if constexpr (sizeof(R) == 4)
      hipLaunchKernelGGL((k_sdiv<R, 1, double, TR>), dim3(rs64_grid(G)), dim3(256), sdiv_lds_bytes(8), st, G.S,
                         G.wl[WL_SDIV], nw);
  } else {
    hipLaunchKernelGGL((k_sdiv<R, 0, R, TR>), dim3(nw), dim3(256), sdiv_lds_bytes(sizeof(R)), st, G.S, G.wl[WL_SDIV], nw);
    if constexpr (sizeof(R) == 4)
      hipLaunchKernelGGL((k_sdiv<R, 0, double, TR>), dim3(rs64_grid(G)), dim3(256), sdiv_lds_bytes(8), st, G.S,
                         G.wl[WL_SDIV], nw);
  }
  HIPCHK(hipGetLastError());
  return 0;
}

// Kernel k (0..9) of the iteration sequence.
template <typename R>
int launch_one(const Group& G, int k) {
  hipStream_t st = G.stream;
  switch (k) {
    case 0:
      if (!G.nwl[WL_SDIV]) break;
      if (G.trac) return launch_sdiv<R, 1>(G);
      return launch_sdiv<R, 0>(G);
    case 1: hipLaunchKernelGGL(k_control, dim3(G.ns), dim3(256), 0, st, G.S, G.ids); break;
    case 2: if (G.nwl[WL_NODE]) hipLaunchKernelGGL(k_gram<R>, dim3(G.nwl[WL_NODE]), dim3(256), 0, st, G.S, G.wl[WL_NODE]); break;
    case 3: hipLaunchKernelGGL(k_alpha, dim3(G.ns), dim3(256), 0, st, G.S, G.ids); break;
    case 6: {
      // z: the fused forward / Green / inverse pass of B0 and 2mu0 plans;
      // for C0 plans the forward pass, the coupled apply, the inverse pass
      int rc = launch_slot<R>(G, 2);
      if (!rc) rc = launch_slot<R>(G, 5);
      if (rc) return rc;
      if (G.nwl[WL_C0])
        hipLaunchKernelGGL(k_green_c0<R>, dim3(G.nwl[WL_C0]), dim3(C0_TILE), 0, st, G.S, G.wl[WL_C0]);
      rc = launch_slot<R>(G, 6);
      if (rc) return rc;
      break;
    }
    default: {
      const int rc = launch_slot<R>(G, k - 4);    // 4 x fwd, 5 y fwd, 7 y inv, 8 x inv
      if (rc) return rc;
      break;
    }
  }
  HIPCHK(hipGetLastError());
  return 0;
}

template <typename R>
int launch_iteration(const Group& G) {
  for (int k = 0; k < FM_N_KERNELS; ++k) {
    const int rc = launch_one<R>(G, k);
    if (rc) return rc;
  }
  return 0;
}

int launch_iterations_eager(const Group& G, int count) {
  for (int i = 0; i < count; ++i) {
    const int rc = G.prec == FM_FP64 ? launch_iteration<double>(G) : launch_iteration<float>(G);
    if (rc) return rc;
  }
  return 0;
}

// Capture `1 << idx` iterations of the group into an executable graph.
int capture_chunk(Group& G, int idx) {
  if (!G.cap) HIPCHK(hipStreamCreateWithFlags(&G.cap, hipStreamNonBlocking));
  const hipStream_t user = G.stream;
  G.stream = G.cap;
  hipError_t e = hipStreamBeginCapture(G.cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) { G.stream = user; return fail(FM_E_HIP, std::string("capture begin: ") + hipGetErrorString(e)); }
  const int rc = launch_iterations_eager(G, 1 << idx);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(G.cap, &graph);
  G.stream = user;
  if (rc) { if (graph) (void)hipGraphDestroy(graph); return rc; }
  if (e != hipSuccess) return fail(FM_E_HIP, std::string("capture end: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(&G.graphs[idx], graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) { G.graphs[idx] = nullptr; return fail(FM_E_HIP, std::string("graph instantiate: ") + hipGetErrorString(e)); }
  return 0;
}

// Enqueue `count` iterations: as a sum of captured power-of-two chunks, or
// eagerly (nine launches each) when graphs are switched off.
int launch_iterations(Group& G, int count) {
  if (!g_use_graphs || G.eager) return launch_iterations_eager(G, count);
  while (count > 0) {
    int idx = 0;
    while (idx + 1 < Group::NGRAPH && (2 << idx) <= count) ++idx;
    if (!G.graphs[idx]) {
      const int rc = capture_chunk(G, idx);
      if (rc) return rc;
    }
    HIPCHK(hipGraphLaunch(G.graphs[idx], G.stream));
    count -= 1 << idx;
  }
  return 0;
}

template <typename R>
int launch_commit_t(fm_plan* p) {
  const Group& G = *p->self;
  if (G.fs) hipLaunchKernelGGL((k_fs_out<R>), dim3(G.nwl[WL_VOX]), dim3(256), 0, G.stream, G.S, G.wl[WL_VOX]);
  else if (G.plastic) hipLaunchKernelGGL((k_commit<R, 1>), dim3(G.nwl[WL_VOX]), dim3(256), 0, G.stream, G.S, G.wl[WL_VOX]);
  else hipLaunchKernelGGL((k_commit<R, 0>), dim3(G.nwl[WL_VOX]), dim3(256), 0, G.stream, G.S, G.wl[WL_VOX]);
  HIPCHK(hipGetLastError());
  return 0;
}

int launch_commit(fm_plan* p) {
  return p->d.prec == FM_FP64 ? launch_commit_t<double>(p) : launch_commit_t<float>(p);
}

// Tick rate of the device wall clock read by the control kernel (kHz).
double wall_clock_khz() {
  static double khz = -1;
  if (khz < 0) {
    int dev = 0, rate = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&rate, hipDeviceAttributeWallClockRate, dev) == hipSuccess)
      khz = rate;
    else
      khz = 0;
  }
  return khz;
}

Ctrl* dev_ctrl(fm_plan* p) { return (Ctrl*)(p->ws + p->lay.ctrl); }
LogEntry* dev_log(fm_plan* p) { return (LogEntry*)(p->ws + p->lay.log); }

// Applied tractions only on Neumann faces of their component (Sec. 2.2).
int check_tractions(const fm_plan_desc& d, const fm_load_step* steps, int n) {
  for (int k = 0; k < n; ++k)
    for (int i = 0; i < 3; ++i)
      for (int a = 0; a < 2; ++a)
        for (int q = 0; q < 3; ++q) {
          const double T = steps[k].traction[i][a][q];
          if (!std::isfinite(T)) return fail(FM_E_INVALID_ARG, "traction is not finite");
          if (T != 0 && d.bc[q][i][a] != FM_BC_NEUMANN)
            return fail(FM_E_BC, "a traction needs a Neumann condition of that component on that face");
        }
  return 0;
}

// Start increment `t` of a plan: upload the control block.
int begin_step(fm_plan* p, const fm_load_step& st, int t, const Ctrl* prev) {
  if (int rc = check_tractions(p->d, &st, 1)) return rc;
  Ctrl c;
  std::memset(&c, 0, sizeof(c));
  c.m = 0;
  c.status = ST_RUNNING;
  c.best_err = INFINITY;
  c.best_m = 0;
  c.step = t;
  c.max_iter = p->d.max_iter;
  c.depth = p->d.aa_depth;
  c.period = p->d.aa_period;
  c.dt = st.dt;
  c.tol = p->d.tol;
  c.lam0 = p->d.lambda0;
  c.mu0 = p->d.mu0;
  c.fp32 = p->d.prec == FM_FP32_MIXED;
  c.rs64 = 0;
  c.has_trac = 0;
  for (int i = 0; i < 3; ++i)
    for (int a = 0; a < 2; ++a)
      for (int q = 0; q < 3; ++q) {
        const double d = 2.0 * st.traction[i][a][q] / p->d.h;
        c.dstar[(i * 2 + a) * 3 + q] = d;
        c.dstar32[(i * 2 + a) * 3 + q] = (float)d;
        c.has_trac |= d != 0;
      }
  for (int q = 0; q < 3; ++q) {
    c.c[q] = st.c[q];
    for (int l = 0; l < 3; ++l) {
      c.G[q * 3 + l] = st.G[q][l];
      for (int m = 0; m < 3; ++m) c.H[(q * 3 + l) * 3 + m] = 0.5 * (st.H[q][l][m] + st.H[q][m][l]);
    }
  }
  for (int i = 0; i < 6; ++i) {
    c.mixed_mask[i] = st.mixed_mask[i] != 0;
    c.mixed_target[i] = st.mixed_target[i];
  }
  if (prev && t > 0) {
    // stress-controlled components continue from the previous increment
    for (int i = 0; i < 6; ++i)
      if (c.mixed_mask[i]) {
        const int a = MI[i], b = MJ[i];
        c.G[a * 3 + b] = prev->G[a * 3 + b];
        c.G[b * 3 + a] = prev->G[b * 3 + a];
      }
  }
  ctrl_fp32_copies(c, p->d.scheme == FM_TETRA2 ? 0.5 * p->d.h : 0.0);
  HIPCHK(hipMemcpyAsync(dev_ctrl(p), &c, sizeof(Ctrl), hipMemcpyHostToDevice, p->stream));
  if (st.ustar) {
    const int64_t n3 = 3 * p->g.Nn;
    hipLaunchKernelGGL(k_add_nodal, dim3(cdiv(n3, 256)), dim3(256), 0, p->stream, (double*)(p->ws + p->lay.uf),
                       st.ustar, 1.0, n3);
    HIPCHK(hipGetLastError());
  }
  p->ustar_cur = st.ustar;
  return 0;
}

// Takes the increment's nodal u* back out of the displacement buffer.
int unfold_ustar(fm_plan* p) {
  if (!p->ustar_cur) return 0;
  const int64_t n3 = 3 * p->g.Nn;
  hipLaunchKernelGGL(k_add_nodal, dim3(cdiv(n3, 256)), dim3(256), 0, p->stream, (double*)(p->ws + p->lay.uf),
                     p->ustar_cur, -1.0, n3);
  HIPCHK(hipGetLastError());
  p->ustar_cur = nullptr;
  return 0;
}

int set_outputs(fm_plan* p, fm_outputs* out) {
  p->sd.out_u = out ? out->u : nullptr;
  p->sd.out_eps = out ? out->eps : nullptr;
  p->sd.out_sig = out ? out->sig : nullptr;
  HIPCHK(hipMemcpyAsync(p->self->S, &p->sd, sizeof(SolveDev), hipMemcpyHostToDevice, p->stream));
  return 0;
}

int finish_step(fm_plan* p, const Ctrl& c, int t, bool last, fm_outputs* out, fm_iter_log* log) {
  // commit internal variables; final increment also writes the field outputs
  if (last && out && (out->eps || out->sig || out->u)) {
    int rc = set_outputs(p, out);
    if (rc) return rc;
  }
  // (nothing to commit for a solve without internal variables unless strain
  // or stress fields are requested)
  if (p->d.with_state || (last && out && (out->eps || out->sig))) {
    const int rc = launch_commit(p);
    if (rc) return rc;
  }
  int rc = 0;
  if (last && out && out->u) {
    hipLaunchKernelGGL(k_out_u, dim3(cdiv(p->g.Nn, 256)), dim3(256), 0, p->stream, p->self->S, 0);
    HIPCHK(hipGetLastError());
  }
  if (last && out && (out->eps || out->sig || out->u)) {
    rc = set_outputs(p, nullptr);
    if (rc) return rc;
  }
  rc = unfold_ustar(p);
  if (rc) return rc;
  if (out && out->macro_sigma)
    for (int i = 0; i < 6; ++i) out->macro_sigma[t * 6 + i] = c.macro[i];
  if (out && out->iters) out->iters[t] = c.m;
  if (out && out->converged) out->converged[t] = c.status == ST_CONVERGED;
  p->total_iters += c.m;
  if (log && log->entries && c.log_count > 0) {
    std::vector<LogEntry> le(c.log_count);
    HIPCHK(hipMemcpyAsync(le.data(), dev_log(p), sizeof(LogEntry) * c.log_count, hipMemcpyDeviceToHost, p->stream));
    HIPCHK(hipStreamSynchronize(p->stream));
    const double khz = wall_clock_khz();
    for (int i = 0; i < c.log_count && log->count < log->capacity; ++i) {
      fm_iter_entry& e = log->entries[log->count++];
      e.step = t; e.iter = i; e.err = le[i].err; e.aa_applied = le[i].aa != 0; e.rs_fp64 = le[i].rs64;
      for (int k = 0; k < 6; ++k) e.macro_sigma[k] = le[i].macro[k];
      e.t_us = khz > 0 ? 1e3 * (double)(int64_t)(le[i].stamp - le[0].stamp) / khz : 0.0;
    }
  }
  return 0;
}

// Iterations to enqueue before the next status read.  From the error decay
// between two reads, the iterations still needed are estimated and three
// quarters of them enqueued (at least one): the solve then rarely enqueues
// iterations past convergence (those return at once, but cost launches),
// at the price of a few more status reads near the end.  Without a usable
// decay estimate the chunk doubles, up to 32.
int next_chunk(const Ctrl& c, double e_prev, int m_prev, int chunk) {
  if (e_prev > 0 && c.err > 0 && c.err < e_prev && c.m > m_prev && c.tol > 0) {
    const double rate = std::pow(c.err / e_prev, 1.0 / (c.m - m_prev));
    const double need = std::log(c.tol / c.err) / std::log(rate);
    if (need > 0 && std::isfinite(need)) return std::max(1, std::min(64, (int)(0.75 * need)));
    return 1;
  }
  return std::min(chunk * 2, 32);
}

int read_ctrl(fm_plan* p, Ctrl& c) {
  HIPCHK(hipMemcpyAsync(&c, dev_ctrl(p), sizeof(Ctrl), hipMemcpyDeviceToHost, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  return 0;
}

}  // namespace

// ---------------------------------------------------------------------------
// Transform-kernel autotuning
// ---------------------------------------------------------------------------
// Candidates for one pass index (all three components): 0 = wavefront kernel
// (pencil length 64E, or 32E / 16E for E in {1, 3}), 1..3 = generic LDS
// kernel with F = Fmax, Fmax/2,
// Fmax/4 transforms per block.  Returns false when the candidate does not
// apply to some component (the pass then keeps its current kernel).
constexpr int N_TUNE = 4;

bool apply_choice(Geometry& g, int pass, int choice) {
  Geometry h = g;
  for (int q = 0; q < 3; ++q) {
    const int axis = pass == 0 || pass == 4 ? 0 : (pass == 2 ? 2 : 1);
    const int L = h.L[q][axis];
    const bool packed = axis == 0 ? true : !h.cplx[q][axis - 1];
    if (choice == 0) {
      int LN;
      const int E = wave_shape(L, LN);
      if (!E) return false;
      if (std::max(std::max(h.s1[q], h.s2[q]) * (int64_t)h.rbytes, h.Nn * (int64_t)8) >= ((int64_t)1 << 32)) return false;
      const int cols = wave_cols(LN, packed);
      size_t bytes = ((size_t)h.n[axis] + 3) * (cols + 1) * 2 * (size_t)h.rbytes;
      if (E == 8) bytes += (size_t)WAVE_PENCILS * WT_SIZE * h.rbytes;
      if (bytes > 150 * 1024) return false;
      h.wE[q][pass] = E;
      h.wN[q][pass] = LN;
      h.cols[q][pass] = cols;
    } else {
      const int Fmax = choose_F(L, h.rbytes, 16);
      if ((Fmax >> (choice - 1)) < 1) return false;
      const int F = Fmax >> (choice - 1);
      if ((generic_radix(L) ? 2 : 1) * (size_t)F * pencil_stride(L) * 2 * h.rbytes > 160 * 1024 - 2048) return false;
      h.wE[q][pass] = 0;
      h.F[q][pass] = F;
      h.cols[q][pass] = packed ? 2 * F : F;
    }
  }
  g = h;
  return true;
}

int rebuild_plan_group(fm_plan* p) {
  fill_pass_descs(p);
  return build_group(*p->self, &p, 1, p->ws + p->lay.group, p->lay.group_bytes, p->stream);
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* fm_last_error(void) { return g_err.c_str(); }

int fm_set_graph_launch(int enable) {
  g_use_graphs = enable != 0;
  return FM_OK;
}

size_t fm_workspace_bytes(const fm_plan_desc* desc) {
  Geometry g;
  if (make_geometry(desc, g)) return 0;
  Layout L;
  make_layout(desc, g, L);
  return L.total;
}

int fm_plan_create(const fm_plan_desc* desc, void* d_workspace, size_t ws_bytes, void* hip_stream, fm_plan** out) {
  if (!out) return fail(FM_E_INVALID_ARG, "null output pointer");
  *out = nullptr;
  std::unique_ptr<fm_plan> p(new fm_plan());
  int rc = make_geometry(desc, p->g);
  if (rc) return rc;
  p->d = *desc;
  make_layout(desc, p->g, p->lay);
  if (!d_workspace) return fail(FM_E_WORKSPACE, "null workspace");
  const uintptr_t base = ((uintptr_t)d_workspace + ALIGN - 1) / ALIGN * ALIGN;
  if (ws_bytes < p->lay.total) return fail(FM_E_WORKSPACE, "workspace smaller than fm_workspace_bytes()");
  p->ws = (char*)base;
  p->stream = (hipStream_t)hip_stream;
  rc = p->d.prec == FM_FP64 ? set_lds_limits<double>() : set_lds_limits<float>();
  if (rc) return rc;
  // device descriptor
  SolveDev& s = p->sd;
  std::memset(&s, 0, sizeof(s));
  const Geometry& g = p->g;
  for (int i = 0; i < 3; ++i) { s.n[i] = g.n[i]; s.N[i] = g.N[i]; }
  s.Nn = g.Nn; s.Nv = g.Nv;
  s.scheme = desc->scheme; s.nppv = g.nppv; s.depth = g.depth; s.has_state = desc->with_state ? 1 : 0;
  for (int q = 0; q < 3; ++q)
    for (int a = 0; a < 3; ++a) s.kinds[q][a] = g.kinds[q][a];
  s.h = desc->h; s.lam0 = desc->lambda0; s.mu0 = desc->mu0;
  char* ws = p->ws;
  s.uf = (double*)(ws + p->lay.uf);
  s.Dring = ws + p->lay.Dring;
  s.dring = ws + p->lay.dring;
  s.mat = (const uint16_t*)(ws + p->lay.mat);
  s.mtab = ws + p->lay.mtab;
  s.mlaw = (const int32_t*)(ws + p->lay.mlaw);
  s.state = desc->with_state ? ws + p->lay.state : nullptr;
  s.sig = (desc->with_state || desc->finite_strain) ? ws + p->lay.sig : nullptr;
  s.fs = desc->finite_strain ? 1 : 0;
  s.ctrl = (Ctrl*)(ws + p->lay.ctrl);
  s.log = (LogEntry*)(ws + p->lay.log);
  s.part_s = (double*)(ws + p->lay.part_s);
  s.part_d = (double*)(ws + p->lay.part_d);
  s.part_g = (double*)(ws + p->lay.part_g);
  s.ntile_s = g.ntile_s; s.ntile_d = g.ntile_d;
  s.mixed_wrap = 0;
  for (int i = 0; i < 3; ++i) {
    s.sd_nt[i] = g.sd_nt[i];
    s.sd_zc = g.sd_zc;
    s.sd_tw = g.sd_tw;
    s.sd_tny = g.sd_tny;
    s.wrap[i] = g.wrap[i];
    for (int q = 0; q < 3; ++q)
      if (g.wrap[i] && g.kinds[q][i] != K_DFT) s.mixed_wrap = 1;
  }
  s.c0 = g.c0;
  if (g.c0) {
    s.c0_cplx = g.cplx[0][2];
    int64_t offC = 0;
    size_t toff = 0;
    for (int a = 0; a < 3; ++a) {
      s.c0_U[a] = g.U[a];
      s.c0_sc[a] = (const double*)(ws + p->lay.c0tab + 8 * toff);
      toff += 2 * (size_t)g.U[a];
    }
    for (int q = 0; q < 3; ++q) {
      s.c0_spec[q] = ws + p->lay.specC + (size_t)g.rbytes * offC;
      offC += g.s3[q];
      int sines = 0;
      for (int a = 0; a < 3; ++a) {
        s.c0_M[q][a] = g.M[q][a];
        s.c0_off[q][a] = g.U[a] - g.M[q][a] == 2 ? 1 : 0;    // DST-I inside the DCT-I frequency set
        sines += g.kinds[q][a] == K_DST1 || g.kinds[q][a] == K_DST3;
      }
      s.c0_phase[q] = sines & 3;
    }
  }
  fill_pass_descs(p.get());
  rc = upload_tables(p.get());
  if (rc) return rc;
  Ctrl c;
  std::memset(&c, 0, sizeof(c));
  c.status = ST_IDLE;
  HIPCHK(hipMemcpyAsync(dev_ctrl(p.get()), &c, sizeof(c), hipMemcpyHostToDevice, p->stream));
  p->self = new Group();
  rc = build_group(*p->self, (fm_plan* const*)&p, 1, ws + p->lay.group, p->lay.group_bytes, p->stream);
  if (rc) { delete p->self; return rc; }
  *out = p.release();
  return FM_OK;
}

void fm_plan_destroy(fm_plan* plan) {
  if (!plan) return;
  delete plan->self;
  delete plan;
}

int64_t fm_plan_total_iterations(const fm_plan* plan) { return plan ? plan->total_iters : -1; }

int fm_set_material(fm_plan* p, const int32_t* d_mat_id, int32_t n_mat, const fm_material* table) {
  if (!p || !d_mat_id || !table || n_mat < 1) return fail(FM_E_INVALID_ARG, "null or empty material arguments");
  if (n_mat > p->d.max_materials) return fail(FM_E_CAPACITY, "more materials than max_materials");
  const size_t R = p->g.rbytes;
  std::vector<int32_t> laws(n_mat);
  std::vector<double> e(MT_STRIDE);
  std::vector<char> tab(R * MT_STRIDE * n_mat);
  for (int i = 0; i < n_mat; ++i) {
    const int law = material_entry(table[i], e.data());
    if (law < 0) return law;
    if ((law == LAW_J2 || law == LAW_CP) && !p->d.with_state)
      return fail(FM_E_UNSUPPORTED, "J2 / CP materials need with_state = 1 in the plan");
    if ((law == LAW_SVK || law == LAW_NEOHOOKE) != (p->d.finite_strain != 0))
      return fail(FM_E_UNSUPPORTED, "finite-strain plans take the SVK and Neo-Hookean laws, small-strain plans the others");
    laws[i] = law;
    for (int k = 0; k < MT_STRIDE; ++k) {
      if (R == 8) ((double*)tab.data())[(size_t)i * MT_STRIDE + k] = e[k];
      else ((float*)tab.data())[(size_t)i * MT_STRIDE + k] = (float)e[k];
    }
  }
  char* ws = p->ws;
  HIPCHK(hipMemcpyAsync(ws + p->lay.mlaw, laws.data(), 4 * n_mat, hipMemcpyHostToDevice, p->stream));
  HIPCHK(hipMemcpyAsync(ws + p->lay.mtab, tab.data(), tab.size(), hipMemcpyHostToDevice, p->stream));
  int* bad = (int*)(ws + p->lay.part_d);   // scratch word
  HIPCHK(hipMemsetAsync(bad, 0, sizeof(int), p->stream));
  hipLaunchKernelGGL(k_mat_convert, dim3(cdiv(p->g.Nv, 256)), dim3(256), 0, p->stream, d_mat_id,
                     (uint16_t*)(ws + p->lay.mat), p->g.Nv, n_mat, bad);
  HIPCHK(hipGetLastError());
  int hbad = 0;
  HIPCHK(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  if (hbad) return fail(FM_E_INVALID_ARG, "material id out of range");
  HIPCHK(hipMemsetAsync(ws + p->lay.uf, 0, 8 * 3 * (size_t)p->g.Nn, p->stream));
  HIPCHK(hipMemsetAsync(ws + p->lay.dring, 0, R * p->g.depth * 3 * (size_t)p->g.Nn, p->stream));
  if (p->d.with_state) {
    HIPCHK(hipMemsetAsync(ws + p->lay.state, 0, R * 7 * p->g.nppv * (size_t)p->g.Nv, p->stream));
    // the stress of the previous iterate, a start of the crystal-plasticity solve
    HIPCHK(hipMemsetAsync(ws + p->lay.sig, 0, R * 6 * p->g.nppv * (size_t)p->g.Nv, p->stream));
  }
  HIPCHK(hipStreamSynchronize(p->stream));
  p->ustar_cur = nullptr;
  p->material_set = true;
  p->n_mat = n_mat;
  return FM_OK;
}

int fm_solve(fm_plan* p, const fm_load_step* steps, int32_t n_steps, fm_outputs* out, fm_iter_log* log) {
  if (!p || !steps || n_steps < 1) return fail(FM_E_INVALID_ARG, "null plan or empty load path");
  if (!p->material_set) return fail(FM_E_STATE, "fm_set_material must be called before fm_solve");
  if (int rc = check_tractions(p->d, steps, n_steps)) return rc;
  set_trac(*p->self, has_traction(steps, n_steps));
  if (log) log->count = 0;
  p->total_iters = 0;
  int result = FM_OK;
  Ctrl prev;
  bool have_prev = false;
  for (int t = 0; t < n_steps; ++t) {
    int rc = begin_step(p, steps[t], t, have_prev ? &prev : nullptr);
    if (rc) return rc;
    Ctrl c;
    int chunk = 4;
    double e_prev = -1.0;
    int m_prev = 0;
    while (true) {
      rc = launch_iterations(*p->self, chunk);
      if (rc) return rc;
      rc = read_ctrl(p, c);
      if (rc) return rc;
      if (c.status != ST_RUNNING) break;
      chunk = next_chunk(c, e_prev, m_prev, chunk);
      e_prev = c.err;
      m_prev = c.m;
    }
    if (c.status == ST_MAXITER) result = FM_W_NOT_CONVERGED;
    rc = finish_step(p, c, t, t == n_steps - 1, out, log);
    if (rc) return rc;
    prev = c;
    have_prev = true;
  }
  HIPCHK(hipStreamSynchronize(p->stream));
  return result;
}

int fm_apply_green(fm_plan* p, const double* d_x, double* d_w) {
  if (!p || !d_x || !d_w) return fail(FM_E_INVALID_ARG, "null argument");
  Ctrl c;
  std::memset(&c, 0, sizeof(c));
  c.status = ST_RUNNING;
  c.depth = p->d.aa_depth;
  c.n_d = 1; c.slot_d[0] = 0; c.alpha[0] = 1.0;
  c.n_b = 0; c.slot_w = 0;
  HIPCHK(hipMemcpyAsync(dev_ctrl(p), &c, sizeof(Ctrl), hipMemcpyHostToDevice, p->stream));
  const int64_t n3 = 3 * p->g.Nn;
  if (p->d.prec == FM_FP64) {
    HIPCHK(hipMemcpyAsync(p->ws + p->lay.Dring, d_x, 8 * n3, hipMemcpyDeviceToDevice, p->stream));
  } else {
    hipLaunchKernelGGL(k_cast_f, dim3(cdiv(n3, 256)), dim3(256), 0, p->stream, d_x, (float*)(p->ws + p->lay.Dring), n3);
  }
  HIPCHK(hipMemsetAsync(p->ws + p->lay.uf, 0, 8 * n3, p->stream));
  const Group& G = *p->self;
  for (int k = 4; k < FM_N_KERNELS; ++k) {
    const int rc = p->d.prec == FM_FP64 ? launch_one<double>(G, k) : launch_one<float>(G, k);
    if (rc) return rc;
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(d_w, p->ws + p->lay.uf, 8 * n3, hipMemcpyDeviceToDevice, p->stream));
  c.status = ST_IDLE;
  HIPCHK(hipMemcpyAsync(dev_ctrl(p), &c, sizeof(Ctrl), hipMemcpyHostToDevice, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  return FM_OK;
}

int fm_residual(fm_plan* p, const fm_load_step* step, const double* d_uf, double* d_D, double* err, double* macro) {
  if (!p || !step || !d_uf || !d_D) return fail(FM_E_INVALID_ARG, "null argument");
  if (!p->material_set) return fail(FM_E_STATE, "fm_set_material must be called first");
  if (int rc = check_tractions(p->d, step, 1)) return rc;
  set_trac(*p->self, has_traction(step, 1));
  int rc = begin_step(p, *step, 0, nullptr);
  if (rc) return rc;
  const int64_t n3 = 3 * p->g.Nn;
  HIPCHK(hipMemcpyAsync(p->ws + p->lay.uf, d_uf, 8 * n3, hipMemcpyDeviceToDevice, p->stream));
  if (step->ustar) {
    hipLaunchKernelGGL(k_add_nodal, dim3(cdiv(n3, 256)), dim3(256), 0, p->stream, (double*)(p->ws + p->lay.uf),
                       step->ustar, 1.0, n3);
    HIPCHK(hipGetLastError());
  }
  p->ustar_cur = step->ustar;   // taken out again below: the buffer ends as d_uf
  const Group& G = *p->self;
  hipStream_t st = p->stream;
  rc = p->d.prec == FM_FP64 ? launch_one<double>(G, 0) : launch_one<float>(G, 0);
  if (rc) return rc;
  hipLaunchKernelGGL(k_control, dim3(1), dim3(256), 0, st, G.S, G.ids);
  HIPCHK(hipGetLastError());
  if (p->d.prec == FM_FP64) {
    HIPCHK(hipMemcpyAsync(d_D, p->ws + p->lay.Dring, 8 * n3, hipMemcpyDeviceToDevice, st));
  } else {
    hipLaunchKernelGGL(k_cast_d, dim3(cdiv(n3, 256)), dim3(256), 0, st, (const float*)(p->ws + p->lay.Dring), d_D, n3);
  }
  Ctrl c;
  rc = read_ctrl(p, c);
  if (rc) return rc;
  if (err) *err = c.err;
  if (macro) for (int i = 0; i < 6; ++i) macro[i] = c.macro[i];
  c.status = ST_IDLE;
  HIPCHK(hipMemcpyAsync(dev_ctrl(p), &c, sizeof(Ctrl), hipMemcpyHostToDevice, st));
  rc = unfold_ustar(p);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(st));
  return FM_OK;
}

}  // extern "C"

namespace {

// A pass slot's work list repeated `reps` times (bucket by bucket), so that
// one launch holds about FILL_BLOCKS blocks; kept in the plan workspace's
// region for it (fewer than 2 FILL_BLOCKS entries per slot).
struct FillList {
  int2* d = nullptr;
  int reps = 1;
  int64_t boff[NBUCKET]{}, bn[NBUCKET]{};
};

int make_fill_list(const Group& G, int slot, int2* region, FillList& f) {
  const int64_t n = G.nwl[WL_PASS0 + slot];
  f.reps = (n == 0 || n >= FILL_BLOCKS) ? 1 : (int)cdiv(FILL_BLOCKS, n);
  if (f.reps == 1) return 0;
  std::vector<int2> h((size_t)n), r;
  HIPCHK(hipMemcpyAsync(h.data(), G.wl[WL_PASS0 + slot], sizeof(int2) * n, hipMemcpyDeviceToHost, G.stream));
  HIPCHK(hipStreamSynchronize(G.stream));
  r.reserve((size_t)n * f.reps);
  for (int b = 0; b < NBUCKET; ++b) {
    f.boff[b] = (int64_t)r.size();
    f.bn[b] = G.bn[slot][b] * f.reps;
    for (int k = 0; k < f.reps; ++k)
      r.insert(r.end(), h.begin() + G.boff[slot][b], h.begin() + G.boff[slot][b] + G.bn[slot][b]);
  }
  if (r.size() > 2 * (size_t)FILL_BLOCKS) return fail(FM_E_INVALID_ARG, "internal: repeated tile list too long");
  f.d = region + (size_t)slot * 2 * FILL_BLOCKS;
  HIPCHK(hipMemcpyAsync(f.d, r.data(), sizeof(int2) * r.size(), hipMemcpyHostToDevice, G.stream));
  // the host vector is released on return: the copy must have completed
  HIPCHK(hipStreamSynchronize(G.stream));
  return 0;
}

// Exchange a slot's work list with its repeated form (called again to undo).
void swap_fill_list(Group& G, int slot, FillList& f) {
  std::swap(G.wl[WL_PASS0 + slot], f.d);
  for (int b = 0; b < NBUCKET; ++b) {
    std::swap(G.boff[slot][b], f.boff[b]);
    std::swap(G.bn[slot][b], f.bn[b]);
  }
}

// Per-kernel mean times of n_iter iterations of *step.  With `fill`, each
// transform pass whose launch would leave the device partly idle runs with
// its tiles repeated until it holds about four blocks per compute unit, and
// its time is divided by the repetitions: the pass's cost when other solves
// fill the device, as in a batch or the server.  The repeated tiles write
// the same outputs (the z pass in place), so the plan's fields hold no
// solution afterwards.
int profile_iterations(fm_plan* p, const fm_load_step* step, int32_t n_iter, double* ms, bool fill) {
  if (!p || !step || n_iter < 1 || !ms) return fail(FM_E_INVALID_ARG, "null argument");
  if (!p->material_set) return fail(FM_E_STATE, "fm_set_material must be called first");
  if (int rc = check_tractions(p->d, step, 1)) return rc;
  set_trac(*p->self, has_traction(step, 1));
  int rc = begin_step(p, *step, 0, nullptr);
  if (rc) return rc;
  Ctrl c;
  rc = read_ctrl(p, c);
  if (rc) return rc;
  c.tol = -1.0;                 // never converged
  c.max_iter = 1 << 30;
  HIPCHK(hipMemcpyAsync(dev_ctrl(p), &c, sizeof(Ctrl), hipMemcpyHostToDevice, p->stream));
  for (int k = 0; k < FM_N_KERNELS; ++k) ms[k] = 0;
  Group& G = *p->self;
  hipStream_t st = p->stream;
  // kernels 4..8 are the pass slots 0..4 (slot 2: the fused z pass)
  FillList fl[5];
  std::vector<hipEvent_t> evs((size_t)n_iter * (FM_N_KERNELS + 1), nullptr);
  auto release = [&]() {
    (void)hipStreamSynchronize(st);
    for (auto& x : evs)
      if (x) { (void)hipEventDestroy(x); x = nullptr; }
  };
  int2* region = (int2*)(p->ws + p->lay.fill);
  for (int sl = 0; fill && sl < 5 && !rc; ++sl) rc = make_fill_list(G, sl, region, fl[sl]);
  for (size_t i = 0; i < evs.size() && !rc; ++i)
    if (hipEventCreate(&evs[i]) != hipSuccess) rc = fail(FM_E_HIP, "event create");
  if (rc) { release(); return rc; }
  // all iterations are enqueued before the first wait, so the stream runs the
  // kernels back to back and each interval is one kernel's execution
  for (int it = 0; it < n_iter && !rc; ++it) {
    hipEvent_t* e = &evs[(size_t)it * (FM_N_KERNELS + 1)];
    if (hipEventRecord(e[0], st) != hipSuccess) rc = fail(FM_E_HIP, "event record");
    for (int k = 0; k < FM_N_KERNELS && !rc; ++k) {
      FillList* f = (k >= 4 && k <= 8 && fl[k - 4].reps > 1) ? &fl[k - 4] : nullptr;
      if (f) swap_fill_list(G, k - 4, *f);
      if (p->d.prec == FM_FP64) rc = launch_one<double>(G, k);
      else rc = launch_one<float>(G, k);
      if (f) swap_fill_list(G, k - 4, *f);
      if (!rc && hipEventRecord(e[k + 1], st) != hipSuccess) rc = fail(FM_E_HIP, "event record");
    }
  }
  if (!rc && hipStreamSynchronize(st) != hipSuccess) rc = fail(FM_E_HIP, "profile synchronize");
  for (int it = 0; it < n_iter && !rc; ++it) {
    hipEvent_t* e = &evs[(size_t)it * (FM_N_KERNELS + 1)];
    for (int k = 0; k < FM_N_KERNELS; ++k) {
      float tms = 0;
      if (hipEventElapsedTime(&tms, e[k], e[k + 1]) != hipSuccess) { rc = fail(FM_E_HIP, "event time"); break; }
      const int reps = (k >= 4 && k <= 8) ? fl[k - 4].reps : 1;
      ms[k] += tms / n_iter / reps;
    }
  }
  release();
  if (rc) return rc;
  c.status = ST_IDLE;
  HIPCHK(hipMemcpyAsync(dev_ctrl(p), &c, sizeof(Ctrl), hipMemcpyHostToDevice, st));
  rc = unfold_ustar(p);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(st));
  return FM_OK;
}

}  // namespace

extern "C" {

int fm_profile_iterations(fm_plan* p, const fm_load_step* step, int32_t n_iter, double* ms) {
  return profile_iterations(p, step, n_iter, ms, false);
}

}  // extern "C"

namespace {
// Transform choices already tuned in this process, per signature: grid,
// per-component transform kinds, precision, scheme, Green operator.
std::mutex g_tune_mu;
std::map<std::string, std::array<int, 5>> g_tune_cache;

std::string tune_key(const fm_plan* p) {
  std::string k;
  for (int i = 0; i < 3; ++i) k += std::to_string(p->g.n[i]) + ",";
  for (int q = 0; q < 3; ++q)
    for (int a = 0; a < 3; ++a) k += std::to_string(p->g.kinds[q][a]);
  k += "/" + std::to_string(p->d.prec) + "/" + std::to_string(p->d.scheme) + "/" + std::to_string(p->d.green);
  return k;
}
}  // namespace

extern "C" {

int fm_autotune(fm_plan* p, const fm_load_step* step, int32_t n_iter, int32_t* choice, double* ms) {
  if (!p || !step || n_iter < 1) return fail(FM_E_INVALID_ARG, "null argument");
  if (!p->material_set) return fail(FM_E_STATE, "fm_set_material must be called first");
  const std::string key = tune_key(p);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      Geometry g = p->g;
      for (int pass = 0; pass < 5; ++pass) {
        if (it->second[pass] >= 0) apply_choice(g, pass, it->second[pass]);
        if (choice) choice[pass] = it->second[pass];
      }
      if (ms)
        for (int i = 0; i < N_TUNE * 5; ++i) ms[i] = -1.0;
      p->g = g;
      return rebuild_plan_group(p);
    }
  }
  const Geometry saved = p->g;
  int best[5];
  double best_ms[5];
  for (int pass = 0; pass < 5; ++pass) {
    best[pass] = -1;
    best_ms[pass] = 1e300;
  }
  double tms[FM_N_KERNELS];
  for (int c = 0; c < N_TUNE; ++c) {
    Geometry g2 = saved;
    bool valid[5], any = false;
    for (int pass = 0; pass < 5; ++pass) any |= (valid[pass] = apply_choice(g2, pass, c));
    for (int pass = 0; pass < 5; ++pass)
      if (ms) ms[c * 5 + pass] = -1.0;
    if (!any) continue;
    p->g = g2;
    int rc = rebuild_plan_group(p);
    if (rc) { p->g = saved; rebuild_plan_group(p); return rc; }
    rc = profile_iterations(p, step, n_iter, tms, true);
    if (rc) { p->g = saved; rebuild_plan_group(p); return rc; }
    for (int pass = 0; pass < 5; ++pass) {
      if (!valid[pass]) continue;
      const double t = tms[4 + pass];
      if (ms) ms[c * 5 + pass] = t;
      if (t < best_ms[pass]) { best_ms[pass] = t; best[pass] = c; }
    }
  }
  Geometry g = saved;
  std::array<int, 5> keep;
  for (int pass = 0; pass < 5; ++pass) {
    if (best[pass] >= 0) apply_choice(g, pass, best[pass]);
    if (choice) choice[pass] = best[pass];
    keep[pass] = best[pass];
  }
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = keep;
  }
  p->g = g;
  return rebuild_plan_group(p);
}

}  // extern "C"

#include "fm_batch.inc"

// ---------------------------------------------------------------------------
// Allocation-free solve (callers that cannot allocate device memory)
// ---------------------------------------------------------------------------
// The workspace of fm_solve_static is this file-scope device array.  In host
// code its name is only a stand-in: the device address of each GPU's copy is
// taken once per device with hipGetSymbolAddress and used everywhere after.
static __device__ __align__(256) char scratch[FM_STATIC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
std::map<int, char*> g_scratch_ptr;   // device index -> address of that device's scratch

int scratch_address(char** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it == g_scratch_ptr.end()) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(FM_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    it = g_scratch_ptr.emplace(dev, (char*)ptr).first;
  }
  *out = it->second;
  return 0;
}
}  // namespace

extern "C" {

int fm_solve_static(const fm_plan_desc* desc, const int32_t* d_mat_id, int32_t n_mat, const fm_material* table,
                    const fm_load_step* steps, int32_t n_steps, fm_outputs* out, fm_iter_log* log,
                    void* hip_stream) {
  if (!desc || !d_mat_id || !table || !steps || n_steps < 1) return fail(FM_E_INVALID_ARG, "null argument");
  const size_t need = fm_workspace_bytes(desc);
  if (!need) return FM_E_INVALID_ARG;
  if (need > (size_t)FM_STATIC_SCRATCH_BYTES)
    return fail(FM_E_CAPACITY, "workspace of " + std::to_string(need) + " bytes exceeds the static scratch of " +
                                   std::to_string((size_t)FM_STATIC_SCRATCH_BYTES) + " bytes");
  char* ws = nullptr;
  int rc = scratch_address(&ws);
  if (rc) return rc;
  fm_plan* p = nullptr;
  rc = fm_plan_create(desc, ws, FM_STATIC_SCRATCH_BYTES, hip_stream, &p);
  if (rc) return rc;
  p->self->eager = true;
  rc = fm_set_material(p, d_mat_id, n_mat, table);
  if (rc == 0) rc = fm_solve(p, steps, n_steps, out, log);
  fm_plan_destroy(p);
  return rc;
}

}  // extern "C"

// Real-space part of an iteration of Algorithm 1 (strain, behaviour law,
// discrete divergence, equilibrium error) and the per-solve control logic
// (convergence test, mixed loading, Anderson acceleration).
//
//  k_sdiv    fused tile kernel: strain at the integration points from the
//            node displacements (HEX1 Eqs. D1HG-D3HG; TETRA2 Eqs.
//            D1T1T2G-D3T1T2G) plus the discrete gradient of the prescribed
//            field, behaviour law, and D_q = sum_l D_l sigma_lq at the kept
//            nodes, with the stress of the mirror voxels obtained from the
//            symmetry / periodicity of the equation's component (Eq.
//            Continuous_der_symmetry_per on the stress columns; for TETRA2
//            the reflection exchanges the two tetrahedra); FP64 block
//            partials of sum_ip w |sigma|^2, sum sigma and sum |D|^2.
//  k_commit  voxel kernel of the end of an increment: internal variables,
//            FP64 strain / stress outputs.
//  k_gram    Gram matrix of the residual history (Anderson, FP64 partials).
//  k_control convergence test (Eq. equilibrium_condition), macroscopic
//            stress, mixed loading update, Anderson schedule.
//  k_alpha   Anderson least squares (FP64 normal equations, Cholesky).
#pragma once
#include "fm_laws.h"

namespace fm {

constexpr int STALL_ITERS = 200;   // iterations without a 1 % better error (stagnation)
constexpr int RS64_STALL = 8;      // same, for an FP32 plan to move its real-space step to FP64
constexpr int RS64_WIN = 12;       // window of the convergence-rate test of that move
constexpr int SPACE_TILE = 1024;   // voxels / nodes per 256-thread block (4 per thread)
constexpr int GRAM_TILE = 4096;    // nodes per 256-thread Gram block (16 per thread)

__device__ __forceinline__ int vidx(int l, int q) {
  // Voigt index of the symmetric pair (l, q): xx yy zz yz xz xy
  return l == q ? l : 6 - l - q;
}

// Per-thread sum of the block partials p[t * N + i] over the tiles
// t = threadIdx.x + k blockDim.x, in increasing k.  Four tiles' loads are
// issued before they are added (the same additions in the same order), so
// a thread waits for one memory round trip per four tiles, not per tile.
template <int N>
__device__ __forceinline__ void sum_tiles(const double* __restrict__ p, int ntile, double (&a)[N]) {
  const int b = blockDim.x;
  int t = threadIdx.x;
  for (; t + 3 * b < ntile; t += 4 * b) {
    double v[4][N];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int i = 0; i < N; ++i) v[u][i] = p[(int64_t)(t + u * b) * N + i];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int i = 0; i < N; ++i) a[i] += v[u][i];
  }
  for (; t < ntile; t += b)
#pragma unroll
    for (int i = 0; i < N; ++i) a[i] += p[(int64_t)t * N + i];
}

template <int N>
__device__ __forceinline__ void block_sum(double (&v)[N], double* out) {
  __shared__ double red[4][N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double x = v[i];
    for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
    v[i] = x;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < N; ++i) red[wv][i] = v[i];
  }
  __syncthreads();
  if (threadIdx.x < N) {
    double s = 0;
    const int nw = (blockDim.x + 63) >> 6;
    for (int k = 0; k < nw; ++k) s += red[k][threadIdx.x];
    out[threadIdx.x] = s;
  }
}

__device__ __forceinline__ bool node_kept(int kind, int n, int j) {
  switch (kind) {
    case K_DFT: return j < n;
    case K_DCT1: return true;
    case K_DST1: return j > 0 && j < n;
    case K_DCT3: return j < n;
    default: return j > 0;
  }
}

// Strain at the integration points of voxel (x, y, z) from the node
// displacements u^f plus the discrete gradient of the prescribed field u*
// (HEX1: one point, all corners, weight (2a_l - 1)/(4h); TETRA2: T1 on the
// even corners and T2 on the odd corners, weight (2a_l - 1)/(2h)).
// FP64: the corner sums are taken in FP64.  FP32: each corner value enters
// as its FP64 difference to corner (0,0,0), rounded once (the stencil
// weights of one point sum to zero, so only differences matter), and the
// rest is FP32.
// Discrete gradient, on one tetrahedron of TETRA2, of the cross terms
// x_a x_b of u*: hc[l][q] enters with - on T1 and + on T2 (0 for HEX1).
template <typename R>
__device__ __forceinline__ void tet_cross_terms(const SolveDev& s, const FM_GLOBAL Ctrl* C, R (&hc)[3][3]) {
  const double c = s.scheme == 1 ? 0.5 * s.h : 0.0;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    hc[0][q] = (R)(c * C->H[(q * 3 + 1) * 3 + 2]);
    hc[1][q] = (R)(c * C->H[(q * 3 + 0) * 3 + 2]);
    hc[2][q] = (R)(c * C->H[(q * 3 + 0) * 3 + 1]);
  }
}

// u* gradient at voxel centres of one column (x, y): gs = gA + gB z_c.
template <typename R>
__device__ __forceinline__ void ustar_grad_column(const SolveDev& s, const FM_GLOBAL Ctrl* C, int x, int y,
                                                  R (&gA)[3][3], R (&gB)[3][3]) {
  const double xc = (x + 0.5) * s.h, yc = (y + 0.5) * s.h;
#pragma unroll
  for (int l = 0; l < 3; ++l)
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const FM_GLOBAL double* H = C->H + (q * 3 + l) * 3;
      gA[l][q] = (R)(C->G[q * 3 + l] + H[0] * xc + H[1] * yc);
      gB[l][q] = (R)H[2];
    }
}

// Corner values of voxel (x, y, z): u[q][c] for FP64; for FP32 the FP64
// difference to corner 0, rounded once (the stencil weights of one point sum
// to zero, so only differences matter).
template <typename R>
__device__ __forceinline__ void voxel_corners(const SolveDev& s, int x, int y, int z, R (&u)[3][8]) {
  const int64_t N0 = s.N[0], N01 = (int64_t)s.N[0] * s.N[1];
  const int64_t base = z * N01 + (int64_t)y * N0 + x;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const FM_GLOBAL double* uq = gconst(s.uf) + q * s.Nn + base;
    const double u0 = uq[0];
    u[q][0] = sizeof(R) == 8 ? (R)u0 : (R)0;
#pragma unroll
    for (int cidx = 1; cidx < 8; ++cidx) {
      const int a = cidx & 1, b = (cidx >> 1) & 1, c = cidx >> 2;
      const double uc = uq[a + b * N0 + c * N01];
      u[q][cidx] = sizeof(R) == 8 ? (R)uc : (R)(uc - u0);
    }
  }
}

// Strain at the integration points of one scheme (SCH 0: HEX1, one point,
// all corners; SCH 1: TETRA2, T1 on the even corners and T2 on the odd
// corners) from the corner values, the u* gradient at the voxel centre and
// the tetrahedron cross-term correction.  FP32 corner values are differences
// to corner 0, which is exactly 0 and left out of the sums.
template <typename R, int SCH, bool ENG = false>
__device__ __forceinline__ void strain_points(const R (&u)[3][8], const R (&gs)[3][3], const R (&hc)[3][3], R f,
                                              R eps[2][6]) {
#pragma unroll
  for (int r = 0; r < (SCH == 1 ? 2 : 1); ++r) {
    R g[3][3];
#pragma unroll
    for (int l = 0; l < 3; ++l)
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        R a = 0;
        bool first = true;
#pragma unroll
        for (int cidx = 0; cidx < 8; ++cidx) {
          const int bit[3] = {cidx & 1, (cidx >> 1) & 1, cidx >> 2};
          const int par = (bit[0] + bit[1] + bit[2]) & 1;
          if (SCH == 1 && par != r) continue;
          if (sizeof(R) == 4 && cidx == 0) continue;
          const R t = bit[l] ? u[q][cidx] : -u[q][cidx];
          a = first ? t : a + t;
          first = false;
        }
        g[l][q] = a * f + gs[l][q];
        if (SCH == 1) g[l][q] += r == 0 ? -hc[l][q] : hc[l][q];
      }
    // ENG: engineering shear strains (twice the tensor components)
    const R hs = ENG ? (R)1 : (R)0.5;
    eps[r][0] = g[0][0]; eps[r][1] = g[1][1]; eps[r][2] = g[2][2];
    eps[r][3] = ENG ? g[1][2] + g[2][1] : hs * (g[1][2] + g[2][1]);
    eps[r][4] = ENG ? g[0][2] + g[2][0] : hs * (g[0][2] + g[2][0]);
    eps[r][5] = ENG ? g[0][1] + g[1][0] : hs * (g[0][1] + g[1][0]);
  }
}

// Strain at the integration points (HEX1: weight (2a_l - 1)/(4h); TETRA2:
// weight (2a_l - 1)/(2h)); the scheme is uniform over a solve, so the branch
// is too.
template <typename R, bool ENG = false>
__device__ __forceinline__ void strain_from_corners(const SolveDev& s, const R (&u)[3][8], const R (&gs)[3][3],
                                                    const R (&hc)[3][3], R eps[2][6]) {
  if (s.scheme == 1)
    strain_points<R, 1, ENG>(u, gs, hc, (R)(0.5 / s.h), eps);
  else
    strain_points<R, 0, ENG>(u, gs, hc, (R)(0.25 / s.h), eps);
}

// Strain at the integration points of voxel (x, y, z).
template <typename R>
__device__ __forceinline__ void voxel_strain(const SolveDev& s, const FM_GLOBAL Ctrl* C, int x, int y, int z, R eps[2][6]) {
  R u[3][8], gA[3][3], gB[3][3], hc[3][3];
  voxel_corners<R>(s, x, y, z, u);
  ustar_grad_column<R>(s, C, x, y, gA, gB);
  tet_cross_terms<R>(s, C, hc);
  const R zc = (R)((z + 0.5) * s.h);
#pragma unroll
  for (int l = 0; l < 3; ++l)
#pragma unroll
    for (int q = 0; q < 3; ++q) gA[l][q] += gB[l][q] * zc;
  strain_from_corners<R>(s, u, gA, hc, eps);
}

// Commit of an increment: behaviour law with the converged strain, internal
// variables stored, FP64 strain / stress outputs.  PL = 0 compiles the
// elastic laws only, PL = 1 all laws.  SIGMA = 1 is the stress pass of an
// iteration of a plastic solve instead: one voxel per thread (four blocks
// per voxel tile), the law with the internal variables of the previous
// increment, the stress into the solve's stress buffer, nothing else written.
template <typename R, int PL, int SIGMA = 0>
__global__ void __launch_bounds__(256, SIGMA ? 2 : 1) k_commit(const SolveDev* __restrict__ S, const int2* __restrict__ work) {
  const int2 w = work[SIGMA ? blockIdx.x / (SPACE_TILE / 256) : blockIdx.x];
  const SolveDev& s = S[w.x];
  const FM_GLOBAL Ctrl* C = gconst(s.ctrl);
  if (SIGMA && (s.sig == nullptr || C->status != ST_RUNNING)) return;
  for (int sub = SIGMA ? (int)(blockIdx.x % (SPACE_TILE / 256)) : 0; sub < SPACE_TILE / 256;
       sub += SIGMA ? SPACE_TILE / 256 : 1) {
    const int64_t v = (int64_t)w.y * SPACE_TILE + sub * 256 + threadIdx.x;
    if (v >= s.Nv) continue;
    const int n0 = s.n[0], n1 = s.n[1];
    const int x = (int)(v % n0);
    const int64_t t = v / n0;
    const int y = (int)(t % n1), z = (int)(t / n1);
    // plastic laws take an FP64 strain: their yield / flow switches must not
    // see the rounding of an FP32 strain, which makes them chatter between
    // iterations and stalls the FP32 solve
    typedef typename std::conditional<PL != 0, double, R>::type E;
    E eps[2][6];
    voxel_strain<E>(s, C, x, y, z, eps);
    const int mt = gconst(s.mat)[v];
    const int law = gconst(s.mlaw)[mt];
    const FM_GLOBAL R* P = gconst((const R*)s.mtab) + (int64_t)mt * MT_STRIDE;
    for (int r = 0; r < s.nppv; ++r) {
      // this point's strain by selects (a runtime index into eps would put
      // the array in scratch memory)
      E er[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) er[k] = r == 0 ? eps[0][k] : eps[1][k];
      R st[7], stn[7];
      FM_GLOBAL R* state = gmut((R*)s.state);
      if (PL && s.has_state) {
#pragma unroll
        for (int k = 0; k < 7; ++k) st[k] = state[((int64_t)k * s.nppv + r) * s.Nv + v];
      } else {
#pragma unroll
        for (int k = 0; k < 7; ++k) st[k] = 0;
      }
      R sig[6];
      if constexpr (PL != 0) {
        // crystal plasticity starts its Newton solve from the point's stress
        // of the previous iteration when that is closer (zero before the first)
        R sp[6];
        const bool warm = s.sig != nullptr && law == LAW_CP;
        if (warm) {
#pragma unroll
          for (int k = 0; k < 6; ++k) sp[k] = gconst((const R*)s.sig)[((int64_t)k * s.nppv + r) * s.Nv + v];
        }
        law_eval_e64<R>(law, P, er, sig, st, stn, C->dt, warm ? sp : nullptr);
      } else {
        law_elastic<R>(law, P, er, sig, st, stn);
      }
      if (SIGMA) {
#pragma unroll
        for (int k = 0; k < 6; ++k) gmut((R*)s.sig)[((int64_t)k * s.nppv + r) * s.Nv + v] = sig[k];
        continue;
      }
      if (PL && s.has_state && (law == LAW_J2 || law == LAW_CP)) {
#pragma unroll
        for (int k = 0; k < 7; ++k) state[((int64_t)k * s.nppv + r) * s.Nv + v] = stn[k];
      }
      if (s.out_eps) {
#pragma unroll
        for (int k = 0; k < 6; ++k) gmut(s.out_eps)[((int64_t)k * s.nppv + r) * s.Nv + v] = (double)er[k];
      }
      if (s.out_sig) {
#pragma unroll
        for (int k = 0; k < 6; ++k) gmut(s.out_sig)[((int64_t)k * s.nppv + r) * s.Nv + v] = (double)sig[k];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Fused stress + divergence of one iteration.
//
// A block owns a tile of SD_TX x SD_TY node columns and sd_zc node layers
// (at most SD_ZC; fewer on small grids and for the costly plastic laws, so
// that there are enough blocks to fill the GPU).
// It marches up the layers: for voxel layer z it evaluates the behaviour law
// on the 32 x 8 voxels that touch the tile (one per thread, the tile plus a
// one-voxel halo; plastic solves read them from their per-voxel stress pass
// instead), sums each voxel column's contributions of layers z-1 and z into
// LDS partials, then forms the divergence at node layer z.  The stress of an
// elastic solve never goes to memory.  Outside the grid a halo voxel holds the periodic image
// along axes periodic for some component, and zero otherwise (see
// node_div for the reflecting faces).  Every voxel's stress enters the
// block partials (sum w |sigma|^2, sum sigma) exactly once, in the tile that
// owns node (x, y, z) of its lower corner; the partials also carry
// sum |D|^2.
// ---------------------------------------------------------------------------
constexpr int SD_TX = 31, SD_TY = 7, SD_ZC = 32;   // node tile (at most SD_ZC layers); voxel tile 32 x 8
constexpr int SD_VT = 256;                          // voxels per layer tile
constexpr int SD_WANT_BLOCKS = 8 * 256;             // stress-divergence tiles that fill the GPU

// Thread box of stress-divergence tile idx: W x H threads over the voxel
// columns of the tile and its one-voxel halo, (W - 1) x (H - 1) node columns
// from (X0, Y0), node layers from Z0.  The x range is cut into 31-node
// tiles; the remainder (fewer than 31 nodes) gets tiles of its own width
// and SD_VT / W rows, so that its threads are not mostly idle.  Threads past
// W x H (SD_VT not a multiple of W) own no voxel and no node.
struct SdBox {
  int X0, Y0, Z0, W, H;
};
__device__ __forceinline__ SdBox sd_box(const SolveDev& s, int idx) {
  const int full = s.sd_nt[0] * s.sd_nt[1];
  const int per = full + s.sd_tny;
  const int z = idx / per, r = idx - z * per;
  SdBox b;
  b.Z0 = z * s.sd_zc;
  if (r < full) {
    b.W = 32; b.H = 8;
    b.X0 = (r % s.sd_nt[0]) * SD_TX;
    b.Y0 = (r / s.sd_nt[0]) * SD_TY;
  } else {
    b.W = s.sd_tw; b.H = SD_VT / s.sd_tw;
    b.X0 = s.sd_nt[0] * SD_TX;
    b.Y0 = (r - full) * (b.H - 1);
  }
  return b;
}

__device__ __forceinline__ int map_vox(int g, int n, int wrap) {
  if (g < 0) return wrap ? n - 1 : 0;
  if (g >= n) return wrap ? min(g - n, n - 1) : n - 1;
  return g;
}

// Faces: a node kept for component q sits on a reflecting face of q only
// where u_q is symmetric (an anti-symmetric face dismisses the node), and
// there each mirror corner contributes exactly what its in-grid image
// contributes (the T1/T2 exchange and the signs of Eq.
// Continuous_der_symmetry_per cancel the flipped stencil sign).  So the
// mirror corners are dropped and the sum is doubled per reflecting face.
// Mirror corners are dropped through halo voxels whose stress is held at
// zero (axes periodic for no component) or, on axes periodic for another
// component, explicitly (z faces in the column partials, x and y faces at
// the node); periodic components read the halo voxel (the periodic image)
// as in the interior.
//
// The divergence at node J sums, over the 8 voxels J - 1 + b (b in {0,1}^3)
// and the directions l, (2 b_l - 1) sigma_lq of the voxel's integration
// point that owns the corner (HEX1: the single point; TETRA2: T1 when
// b0 + b1 + b2 is odd, T2 when even).  The two z layers are summed first,
// per voxel column: column (x, y) holds for each offset (b0, b1) and each q
// the partial over b2 and l, from its own stresses of layers J2 - 1 and J2
// (kept in registers), with the mirror corners of the z faces dropped; the
// node then adds the partials of its four columns, dropping those of mirror
// corners on the x and y faces.  sp / sc: stresses of the column's voxel in
// layers J2 - 1 and J2, [point][Voigt] (HEX1: the point in both slots).
template <typename R, bool FACE>
__device__ __forceinline__ void column_partials(const SolveDev& s, const R (&sp)[2][6], const R (&sc)[2][6], int J2,
                                                R* __restrict__ P) {
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    // a / b: S_lq of the points (index r) of the voxel below (b2 = 0) and
    // above (b2 = 1) the node layer; on a z face, the mirror corners of a
    // component not periodic along z are dropped
    bool drop0 = false, drop1 = false;
    if constexpr (FACE) {
      const bool zf = s.wrap[2] && s.kinds[q][2] != K_DFT;
      drop0 = zf && J2 == 0;
      drop1 = zf && J2 == s.n[2];
    }
    R a[2][3], b[2][3];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        a[r][l] = drop0 ? (R)0 : sp[r][vidx(l, q)];
        b[r][l] = drop1 ? (R)0 : sc[r][vidx(l, q)];
      }
    // offsets (b0, b1) with b0 + b1 even take point 1 below and point 0
    // above, odd ones point 0 below and point 1 above (HEX1: one point);
    // the partial is sum_l (2 b_l - 1) S_lq over the two voxels
    const R Xe = a[1][0] + b[0][0], Ye = a[1][1] + b[0][1], Ze = b[0][2] - a[1][2];
    const R Xo = a[0][0] + b[1][0], Yo = a[0][1] + b[1][1], Zo = b[1][2] - a[0][2];
    const R Se = Xe + Ye, To = Xo - Yo;
    P[(q * 4 + 0) * SD_VT] = Ze - Se;     // (b0, b1) = (0, 0)
    P[(q * 4 + 3) * SD_VT] = Ze + Se;     // (1, 1)
    P[(q * 4 + 1) * SD_VT] = Zo + To;     // (1, 0)
    P[(q * 4 + 2) * SD_VT] = Zo - To;     // (0, 1)
  }
}

// Per-node constants of the x-y position: the factor of each component
// (1/(4h), doubled per reflecting x or y face, 0 where the node is not kept
// along x or y) and the mirror-corner drops of those faces, bit
// (q * 4 + b1 * 2 + b0) set when column offset (b0, b1) is a mirror corner
// of an axis periodic for another component.
template <typename R>
struct NodeXY {
  R fq[3];
  int drop;
};

// D* of a uniform traction T on a Neumann face of u_q (Sec. 2.2): the
// applied stress P* is twice the face value on the face's mirror voxels and
// zero in the grid, so at every kept node of that face the stencil sums four
// mirror voxels of weight 1/(4h) (HEX1; TETRA2 gives the same total), with
// signs that make D*_q = 2 T_q / h on both faces of an axis.  The control
// block holds 2 T / h per [axis][face][component].
template <typename R>
__device__ __forceinline__ R dstar(const FM_GLOBAL Ctrl* C, int i, int a, int q) {
  if constexpr (sizeof(R) == 4) return C->dstar32[(i * 2 + a) * 3 + q];
  else return (R)C->dstar[(i * 2 + a) * 3 + q];
}

// D*_q of the applied tractions at node (J0, J1, J2): the sum over the
// loaded faces the node lies on (read only when some face is loaded).
template <typename R>
__device__ __forceinline__ R node_dstar(const SolveDev& s, const FM_GLOBAL Ctrl* C, int J0, int J1, int J2, int q) {
  R t = 0;
  if (J0 == 0) t += dstar<R>(C, 0, 0, q);
  if (J0 == s.n[0]) t += dstar<R>(C, 0, 1, q);
  if (J1 == 0) t += dstar<R>(C, 1, 0, q);
  if (J1 == s.n[1]) t += dstar<R>(C, 1, 1, q);
  if (J2 == 0) t += dstar<R>(C, 2, 0, q);
  if (J2 == s.n[2]) t += dstar<R>(C, 2, 1, q);
  return t;
}

template <typename R>
__device__ __forceinline__ NodeXY<R> node_xy(const SolveDev& s, int J0, int J1) {
  NodeXY<R> r;
  r.drop = 0;
  const int J[2] = {J0, J1};
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    R fq = (R)(0.25 / s.h);
    bool kept = true;
    int side[2] = {0, 0};                 // bit b: mirror side b dropped
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      kept = kept && node_kept(s.kinds[q][i], s.n[i], J[i]);
      const bool face = s.kinds[q][i] != K_DFT && (J[i] == 0 || J[i] == s.n[i]);
      if (face) fq *= (R)2;
      if (face && s.wrap[i]) side[i] = J[i] == 0 ? 1 : 2;
    }
    r.fq[q] = kept ? fq : (R)0;
#pragma unroll
    for (int b1 = 0; b1 < 2; ++b1)
#pragma unroll
      for (int b0 = 0; b0 < 2; ++b0)
        if (((side[0] >> b0) & 1) || ((side[1] >> b1) & 1)) r.drop |= 1 << (q * 4 + b1 * 2 + b0);
  }
  return r;
}

// Divergence at the node of layer J2 (z factor fz per component: doubling on
// a reflecting z face, 0 where not kept along z) from the column partials of
// its four voxel columns; D written through Dn (this node in component 0).
template <typename CT, typename R, int TR, bool DROP>
__device__ __forceinline__ void node_div(const CT* __restrict__ P, int lx, int ly, int TW, const NodeXY<CT>& nxy,
                                         const CT (&fz)[3], FM_GLOBAL R* Dn, int64_t Nn, CT& accD,
                                         const SolveDev& s, const FM_GLOBAL Ctrl* C, int J0, int J1, int J2) {
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    CT D = 0;
#pragma unroll
    for (int b1 = 0; b1 < 2; ++b1)
#pragma unroll
      for (int b0 = 0; b0 < 2; ++b0) {
        const CT t = P[(q * 4 + b1 * 2 + b0) * SD_VT + (ly + b1) * TW + (lx + b0)];
        if constexpr (DROP) D += ((nxy.drop >> (q * 4 + b1 * 2 + b0)) & 1) ? (CT)0 : t;
        else D += t;
      }
    const CT f = nxy.fq[q] * fz[q];
    CT Dq = D * f;
    if (TR && f != (CT)0) Dq += node_dstar<CT>(s, C, J0, J1, J2, q);
    accD += Dq * Dq;
    Dn[q * Nn] = (R)Dq;
  }
}

// Bytes of dynamic LDS of k_sdiv.
__host__ __device__ inline size_t sdiv_lds_bytes(int rbytes) { return (size_t)2 * 12 * SD_VT * rbytes; }

// PL = 1: the group holds solves with internal variables, whose stresses
// come from the stress pass (k_commit with SIGMA = 1); the law evaluated here
// is elastic.  R is the storage type of the solve's fields (residual ring,
// material table, stress buffer), CT the type the kernel computes in.  FP32
// solves launch both the CT = float kernel and the CT = double one; the
// control block's rs64 flag selects which of the two does the work (the
// FP64 one once the FP32 residual has stalled at its rounding floor).
template <typename R, int PL, typename CT, int TR>
__device__ __forceinline__ void sdiv_tile(const SolveDev* __restrict__ S, const int2 w) {
  const SolveDev& s = S[w.x];
  const FM_GLOBAL Ctrl* C = gconst(s.ctrl);
  if (C->status != ST_RUNNING) return;
  if (sizeof(R) == 4 && (C->rs64 != 0) != (sizeof(CT) == 8)) return;
  extern __shared__ __align__(16) char smem[];
  CT* sl = (CT*)smem;                                  // column partials [2][12][SD_VT]
  const SdBox bx = sd_box(s, w.y);
  const int X0 = bx.X0, Y0 = bx.Y0, Z0 = bx.Z0, TW = bx.W;
  const int Z1 = min(Z0 + s.sd_zc, s.N[2]);
  const int lx = (int)threadIdx.x % TW, ly = (int)threadIdx.x / TW;
  const int n0 = s.n[0], n1 = s.n[1], n2 = s.n[2];
  const int gx = X0 - 1 + lx, gy = Y0 - 1 + ly;
  const int vx = map_vox(gx, n0, s.wrap[0]), vy = map_vox(gy, n1, s.wrap[1]);
  const bool own_xy = lx >= 1 && ly >= 1 && ly < bx.H && gx < n0 && gy < n1;
  const bool zero_xy = (!s.wrap[0] && (gx < 0 || gx >= n0)) || (!s.wrap[1] && (gy < 0 || gy >= n1));
  const int J0 = X0 + lx, J1 = Y0 + ly;
  const bool has_node = lx < TW - 1 && ly < bx.H - 1 && J0 < s.N[0] && J1 < s.N[1];
  const FM_GLOBAL uint16_t* mat = gconst(s.mat);
  const CT wip = (CT)1 / (CT)s.nppv;
  // per-thread partials in CT (each thread sums at most 2 (sd_zc + 1) points),
  // FP64 across the block
  CT acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  // u* gradient of this voxel column: gA + gB z_c.  FP32: from the uniform
  // FP32 copies in the control block (gB and the cross terms stay scalar).
  CT gA[3][3], gB[3][3], hc[3][3];
  if constexpr (sizeof(CT) == 4) {
    // read before any store, so that the uniform values can live in scalars
    const float xc = (float)((vx + 0.5) * s.h), yc = (float)((vy + 0.5) * s.h);
#pragma unroll
    for (int l = 0; l < 3; ++l)
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        gA[l][q] = C->g32[q * 3 + l] + C->h32[(q * 3 + l) * 3] * xc + C->h32[(q * 3 + l) * 3 + 1] * yc;
        gB[l][q] = C->h32[(q * 3 + l) * 3 + 2];
        hc[l][q] = C->hc32[l * 3 + q];
      }
  } else {
    ustar_grad_column<CT>(s, C, vx, vy, gA, gB);
    tet_cross_terms<CT>(s, C, hc);
  }
  // stresses of this column's voxel in the previous and current layer
  // ([point][Voigt], zero on halo voxels; HEX1 duplicates its point)
  CT sprev[2][6], scur[2][6];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int k = 0; k < 6; ++k) sprev[r][k] = scur[r][k] = 0;
  const NodeXY<CT> nxy = node_xy<CT>(s, J0, J1);
  // x-y mirror drops occur only on the faces of axes periodic for another
  // component: waves without any take the plain four-column sums
  const bool wave_drop = __any(nxy.drop != 0);
  // plastic solves read the stresses of the per-voxel stress pass
  const bool from_buf = PL && s.sig != nullptr;
  // FP32 corner carry: top corner 4 (FP64) and corners 5-7 minus it, per component
  double cu4[3] = {0, 0, 0};
  CT cdt[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  int vz_prev = -2;
  const int64_t N01 = (int64_t)s.N[0] * s.N[1];
  FM_GLOBAL R* Dcol = gmut((R*)s.Dring) + (int64_t)(C->m % s.depth) * 3 * s.Nn + (int64_t)J1 * s.N[0] + J0;
  int mt_cur = mat[((int64_t)map_vox(Z0 - 1, n2, s.wrap[2]) * n1 + vy) * n0 + vx];
  for (int zl = Z0 - 1; zl < Z1; ++zl) {
    // material of the next voxel layer, fetched one layer ahead
    // (unconditional: the last layer reads a valid voxel it does not use, so the
    // load needs no branch and its wait can sink to the end of the layer)
    const uint16_t mt_next = mat[((int64_t)map_vox(zl + 1, n2, s.wrap[2]) * n1 + vy) * n0 + vx];
    {
      const int vz = map_vox(zl, n2, s.wrap[2]);
      const int law = gconst(s.mlaw)[mt_cur];
      // halo voxels across faces of axes periodic for no component hold zero
      // stress: their elastic law reads the all-zero entry
      const bool zero_halo = zero_xy || (!s.wrap[2] && (zl < 0 || zl >= n2));
      const FM_GLOBAL R* P = (!from_buf && zero_halo) ? zero_material<R>()
                                                      : gconst((const R*)s.mtab) + (int64_t)mt_cur * MT_STRIDE;
      CT eps[2][6];
      if (!from_buf) {
        CT u[3][8], gs[3][3];
        if constexpr (sizeof(CT) == 4) {
          // FP32: FP64 differences to corner 0, with the bottom face taken
          // from the previous layer's top face when the layers are adjacent
          // (its differences to its own corner 0 formed from the rounded
          // top-face differences)
          const bool carry = zl >= Z0 && vz == vz_prev + 1;
          const int64_t base = (int64_t)vz * N01 + (int64_t)vy * s.N[0] + vx;
#pragma unroll
          for (int q = 0; q < 3; ++q) {
            const FM_GLOBAL double* uq = gconst(s.uf) + q * s.Nn + base;
            double u0;
            if (carry) {
              u0 = cu4[q];
#pragma unroll
              for (int c = 1; c < 4; ++c) u[q][c] = cdt[q][c - 1];
            } else {
              u0 = uq[0];
#pragma unroll
              for (int c = 1; c < 4; ++c) u[q][c] = (CT)(uq[(c & 1) + (c >> 1) * s.N[0]] - u0);
            }
            u[q][0] = 0;
            double top[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) top[c] = uq[(c & 1) + (c >> 1) * s.N[0] + N01];
#pragma unroll
            for (int c = 0; c < 4; ++c) u[q][4 + c] = (CT)(top[c] - u0);
            cu4[q] = top[0];
#pragma unroll
            for (int c = 1; c < 4; ++c) cdt[q][c - 1] = u[q][4 + c] - u[q][4];
          }
          vz_prev = vz;
        } else {
          voxel_corners<CT>(s, vx, vy, vz, u);
        }
        const CT zc = (CT)((vz + 0.5) * s.h);
#pragma unroll
        for (int l = 0; l < 3; ++l)
#pragma unroll
          for (int q = 0; q < 3; ++q) gs[l][q] = gA[l][q] + gB[l][q] * zc;
        strain_from_corners<CT, true>(s, u, gs, hc, eps);
      }
      // the Voigt stiffness of the voxel (read for every law, outside the
      // law's branch, so that the loads issue together)
      CT cv[21];
      if (!from_buf) {
#pragma unroll
        for (int k = 0; k < 21; ++k) cv[k] = (CT)P[MT_VOIGT + k];
      }
      const int64_t v = ((int64_t)vz * n1 + vy) * n0 + vx;
      const bool own = own_xy && zl >= Z0 && zl < n2;
      // the stresses of the voxel's points (one law branch per voxel, so the
      // material entry is read once for both points)
      CT sig2[2][6];
      if (from_buf) {
#pragma unroll
        for (int r = 0; r < 2; ++r)
          if (r < s.nppv)
#pragma unroll
            for (int k = 0; k < 6; ++k) sig2[r][k] = gconst((const R*)s.sig)[((int64_t)k * s.nppv + r) * s.Nv + v];
      } else if (s.nppv == 2) {
        // solves without internal variables: elastic laws only
        law_elastic_pts_eng<CT, 2>(law, cv, eps, sig2);
      } else {
        law_elastic_pts_eng<CT, 1>(law, cv, eps, sig2);
      }
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        if (r >= s.nppv) break;
        const CT (&sig)[6] = sig2[r];
        // (stresses read from the stress buffer are zeroed here)
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          const CT val = (from_buf && zero_halo) ? (CT)0 : sig[k];
          scur[0][k] = r == 0 ? val : scur[0][k];
          scur[1][k] = r == 0 ? val : (r == 1 ? val : scur[1][k]);
        }
        if (own) {
          CT n2s = 0;
#pragma unroll
          for (int k = 0; k < 6; ++k) {
            n2s += (k < 3 ? (CT)1 : (CT)2) * sig[k] * sig[k];
            acc[1 + k] += wip * sig[k];
          }
          acc[0] += wip * n2s;
        }
      }
    }
    if (zl >= Z0) {
      // the partials of consecutive layers alternate between two buffers: a
      // layer's writes come after the barrier of the layer before, which
      // every thread passes only once it has read the buffer two layers back
      CT* slb = sl + (zl & 1) * 12 * SD_VT;
      if (zl == 0 || zl == n2) column_partials<CT, true>(s, sprev, scur, zl, slb + threadIdx.x);
      else column_partials<CT, false>(s, sprev, scur, zl, slb + threadIdx.x);
      CT fz[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const bool face = s.kinds[q][2] != K_DFT && (zl == 0 || zl == n2);
        fz[q] = node_kept(s.kinds[q][2], n2, zl) ? (face ? (CT)2 : (CT)1) : (CT)0;
      }
      __syncthreads();
      if (has_node) {
        if (wave_drop)
          node_div<CT, R, TR, true>(slb, lx, ly, TW, nxy, fz, Dcol + (int64_t)zl * N01, s.Nn, acc[7], s, C, X0 + lx,
                                    Y0 + ly, zl);
        else
          node_div<CT, R, TR, false>(slb, lx, ly, TW, nxy, fz, Dcol + (int64_t)zl * N01, s.Nn, acc[7], s, C, X0 + lx,
                                     Y0 + ly, zl);
      }
    }
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int k = 0; k < 6; ++k) sprev[r][k] = scur[r][k];
    mt_cur = mt_next;
  }
  __shared__ double outp[8];
  double accd[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) accd[i] = (double)acc[i];
  block_sum<8>(accd, outp);
  __syncthreads();
  if (threadIdx.x < 8) gmut(s.part_s)[(int64_t)w.y * NPART_S + threadIdx.x] = outp[threadIdx.x];
}

// FP32 elastic groups: the same tile as sdiv_tile, software-pipelined over
// the voxel layers.  The FP64 top face of layer z + 1's voxel is loaded as
// soon as layer z's corner differences are formed, its Voigt stiffness and
// law (and the material id of layer z + 2) as soon as layer z's law has
// been evaluated, so that their latency overlaps the rest of the layer
// (vector-memory loads complete in order, and a wait for an earlier load
// leaves the later ones in flight).  The bottom face of a
// voxel comes from the previous layer's top face (carry) or, on the first
// layer of the tile and across a periodic wrap, from a load of its own.
template <typename R, int TR>
__device__ __forceinline__ void sdiv_tile_f32(const SolveDev* __restrict__ S, const int2 w) {
  typedef float CT;
  const SolveDev& s = S[w.x];
  const FM_GLOBAL Ctrl* C = gconst(s.ctrl);
  if (C->status != ST_RUNNING) return;
  if (C->rs64 != 0) return;
  extern __shared__ __align__(16) char smem[];
  CT* sl = (CT*)smem;                                  // column partials [2][12][SD_VT]
  const SdBox bx = sd_box(s, w.y);
  const int X0 = bx.X0, Y0 = bx.Y0, Z0 = bx.Z0, TW = bx.W;
  const int Z1 = min(Z0 + s.sd_zc, s.N[2]);
  const int lx = (int)threadIdx.x % TW, ly = (int)threadIdx.x / TW;
  const int n0 = s.n[0], n1 = s.n[1], n2 = s.n[2];
  const int gx = X0 - 1 + lx, gy = Y0 - 1 + ly;
  const int vx = map_vox(gx, n0, s.wrap[0]), vy = map_vox(gy, n1, s.wrap[1]);
  const bool own_xy = lx >= 1 && ly >= 1 && ly < bx.H && gx < n0 && gy < n1;
  const bool zero_xy = (!s.wrap[0] && (gx < 0 || gx >= n0)) || (!s.wrap[1] && (gy < 0 || gy >= n1));
  const int J0 = X0 + lx, J1 = Y0 + ly;
  const bool has_node = lx < TW - 1 && ly < bx.H - 1 && J0 < s.N[0] && J1 < s.N[1];
  const FM_GLOBAL uint16_t* mat = gconst(s.mat);
  const FM_GLOBAL int* mlaw = gconst(s.mlaw);
  const FM_GLOBAL R* mtab = gconst((const R*)s.mtab);
  const CT wip = (CT)1 / (CT)s.nppv;
  CT acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  CT gA[3][3], gB[3][3], hc[3][3];
  {
    const float xc = (float)((vx + 0.5) * s.h), yc = (float)((vy + 0.5) * s.h);
#pragma unroll
    for (int l = 0; l < 3; ++l)
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        gA[l][q] = C->g32[q * 3 + l] + C->h32[(q * 3 + l) * 3] * xc + C->h32[(q * 3 + l) * 3 + 1] * yc;
        gB[l][q] = C->h32[(q * 3 + l) * 3 + 2];
        hc[l][q] = C->hc32[l * 3 + q];
      }
  }
  CT sprev[2][6], scur[2][6];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int k = 0; k < 6; ++k) sprev[r][k] = scur[r][k] = 0;
  const NodeXY<CT> nxy = node_xy<CT>(s, J0, J1);
  const bool wave_drop = __any(nxy.drop != 0);
  const int64_t N0 = s.N[0], N01 = (int64_t)s.N[0] * s.N[1], Nn = s.Nn;
  const FM_GLOBAL double* uf = gconst(s.uf);
  FM_GLOBAL R* Dcol = gmut((R*)s.Dring) + (int64_t)(C->m % s.depth) * 3 * s.Nn + (int64_t)J1 * s.N[0] + J0;
  const int64_t col = (int64_t)vy * n0 + vx;            // voxel column
  const int64_t ncol = (int64_t)vy * N0 + vx;           // its corner-0 node column
  auto vz_of = [&](int z) { return map_vox(z, n2, s.wrap[2]); };
  auto halo_z = [&](int z) { return !s.wrap[2] && (z < 0 || z >= n2); };
  // stage of the layer being computed: raw top face, stiffness, law
  double top[3][4];
  CT cv[21];
  int law;
  auto load_top = [&](int vz, double (&t)[3][4]) {
    const FM_GLOBAL double* b = uf + (int64_t)(vz + 1) * N01 + ncol;
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
      for (int c = 0; c < 4; ++c) t[q][c] = b[q * Nn + (c & 1) + (c >> 1) * N0];
  };
  auto load_law = [&](int z, int mt, CT (&c)[21], int& lw) {
    const FM_GLOBAL R* P = (zero_xy || halo_z(z)) ? zero_material<R>() : mtab + (int64_t)mt * MT_STRIDE;
#pragma unroll
    for (int k = 0; k < 21; ++k) c[k] = (CT)P[MT_VOIGT + k];
    lw = mlaw[mt];
  };
  // prologue: the first layer's stage, the next layer's material
  int vz = vz_of(Z0 - 1);
  {
    const int mt0 = mat[(int64_t)vz * n1 * n0 + col];
    load_top(vz, top);
    load_law(Z0 - 1, mt0, cv, law);
  }
  int mt1 = mat[(int64_t)vz_of(Z0) * n1 * n0 + col];
  double cu4[3] = {0, 0, 0};
  CT cdt[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  int vz_prev = -2;
  for (int zl = Z0 - 1; zl < Z1; ++zl) {
    // corner differences of this layer's voxel (FP64, rounded once)
    CT u[3][8];
    const bool carry = vz == vz_prev + 1;
    if (!carry) {
      const FM_GLOBAL double* b = uf + (int64_t)vz * N01 + ncol;
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        double bt[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) bt[c] = b[q * Nn + (c & 1) + (c >> 1) * N0];
        cu4[q] = bt[0];
#pragma unroll
        for (int c = 1; c < 4; ++c) cdt[q][c - 1] = (CT)(bt[c] - bt[0]);
      }
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const double u0 = cu4[q];
      u[q][0] = 0;
#pragma unroll
      for (int c = 1; c < 4; ++c) u[q][c] = cdt[q][c - 1];
#pragma unroll
      for (int c = 0; c < 4; ++c) u[q][4 + c] = (CT)(top[q][c] - u0);
      cu4[q] = top[q][0];
#pragma unroll
      for (int c = 1; c < 4; ++c) cdt[q][c - 1] = u[q][4 + c] - u[q][4];
    }
    vz_prev = vz;
    // issue the next layer's top face (the last layer reads valid data it
    // does not use)
    const int vzn = vz_of(zl + 1);
    load_top(vzn, top);
    {
      CT eps[2][6], gs[3][3];
      const CT zc = (CT)((vz + 0.5) * s.h);
#pragma unroll
      for (int l = 0; l < 3; ++l)
#pragma unroll
        for (int q = 0; q < 3; ++q) gs[l][q] = gA[l][q] + gB[l][q] * zc;
      strain_from_corners<CT, true>(s, u, gs, hc, eps);
      const bool own = own_xy && zl >= Z0 && zl < n2;
      CT sig2[2][6];
      if (s.nppv == 2) law_elastic_pts_eng<CT, 2>(law, cv, eps, sig2);
      else law_elastic_pts_eng<CT, 1>(law, cv, eps, sig2);
      // and, the stiffness consumed, the next layer's stiffness and law and
      // the material of the layer after it
      load_law(zl + 1, mt1, cv, law);
      mt1 = mat[(int64_t)vz_of(zl + 2) * n1 * n0 + col];
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        if (r >= s.nppv) break;
        const CT (&sig)[6] = sig2[r];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          scur[0][k] = r == 0 ? sig[k] : scur[0][k];
          scur[1][k] = sig[k];
        }
        if (own) {
          CT n2s = 0;
#pragma unroll
          for (int k = 0; k < 6; ++k) {
            n2s += (k < 3 ? (CT)1 : (CT)2) * sig[k] * sig[k];
            acc[1 + k] += wip * sig[k];
          }
          acc[0] += wip * n2s;
        }
      }
    }
    if (zl >= Z0) {
      CT* slb = sl + (zl & 1) * 12 * SD_VT;
      if (zl == 0 || zl == n2) column_partials<CT, true>(s, sprev, scur, zl, slb + threadIdx.x);
      else column_partials<CT, false>(s, sprev, scur, zl, slb + threadIdx.x);
      CT fz[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const bool face = s.kinds[q][2] != K_DFT && (zl == 0 || zl == n2);
        fz[q] = node_kept(s.kinds[q][2], n2, zl) ? (face ? (CT)2 : (CT)1) : (CT)0;
      }
      __syncthreads();
      if (has_node) {
        if (wave_drop)
          node_div<CT, R, TR, true>(slb, lx, ly, TW, nxy, fz, Dcol + (int64_t)zl * N01, s.Nn, acc[7], s, C, X0 + lx,
                                    Y0 + ly, zl);
        else
          node_div<CT, R, TR, false>(slb, lx, ly, TW, nxy, fz, Dcol + (int64_t)zl * N01, s.Nn, acc[7], s, C, X0 + lx,
                                     Y0 + ly, zl);
      }
    }
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int k = 0; k < 6; ++k) sprev[r][k] = scur[r][k];
    vz = vzn;
  }
  __shared__ double outp[8];
  double accd[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) accd[i] = (double)acc[i];
  block_sum<8>(accd, outp);
  __syncthreads();
  if (threadIdx.x < 8) gmut(s.part_s)[(int64_t)w.y * NPART_S + threadIdx.x] = outp[threadIdx.x];
}

// The FP64 variant of an FP32 group is launched every iteration but works
// only for solves near their FP32 rounding floor: it runs as a few blocks
// per compute unit walking the tile list, so that it costs a short dispatch
// when no solve needs it.  Block b owns the items b, b + G, b + 2G, ...
// (G = gridDim.x); it checks 256 of them at once (one per thread: status
// and flag of the item's solve) and then transforms only those that need
// the FP64 step, so that a batch whose solves mostly run in FP32 costs one
// round of flag loads per 256 items instead of one per item.
// TR = 1 adds the applied-traction term D* at the loaded faces (groups whose
// load paths carry tractions; the common kernel carries no traction code).
template <typename R, int PL, typename CT = R, int TR = 0>
__global__ void __launch_bounds__(256, sizeof(CT) == 8 ? 1 : (sizeof(R) == 4 && PL == 0 ? 3 : 4))
    k_sdiv(const SolveDev* __restrict__ S, const int2* __restrict__ work, int nwork) {
  if constexpr (sizeof(R) == 4 && sizeof(CT) == 4 && PL == 0) {
    sdiv_tile_f32<R, TR>(S, work[blockIdx.x]);
  } else if constexpr (sizeof(R) == 4 && sizeof(CT) == 8) {
    __shared__ int2 todo[256];
    __shared__ int ntodo;
    const int64_t G = gridDim.x;
    for (int64_t i0 = blockIdx.x; i0 < nwork; i0 += G * 256) {
      if (threadIdx.x == 0) ntodo = 0;
      __syncthreads();
      const int64_t i = i0 + (int64_t)threadIdx.x * G;
      if (i < nwork) {
        const int2 w = work[i];
        const FM_GLOBAL Ctrl* C = gconst(S[w.x].ctrl);
        if (C->status == ST_RUNNING && C->rs64 != 0) todo[atomicAdd(&ntodo, 1)] = w;
      }
      __syncthreads();
      const int nt = ntodo;
      for (int k = 0; k < nt; ++k) {
        sdiv_tile<R, PL, CT, TR>(S, todo[k]);
        __syncthreads();
      }
      __syncthreads();   // every thread has read ntodo before the next reset
    }
  } else {
    sdiv_tile<R, PL, CT, TR>(S, work[blockIdx.x]);
  }
}

// Gram matrix of the residual window, on Anderson steps only.  Dismissed
// nodes hold D = 0, so every node enters without a mask.  Each thread takes
// GRAM_TILE / 256 nodes in chunks of four, issuing all of a component's
// loads in a chunk before using them; products are summed per chunk in R,
// across chunks and the block in FP64.  The large tile keeps the
// block partials few: one block per solve reduces them (k_alpha).
template <typename R>
__global__ void __launch_bounds__(256) k_gram(const SolveDev* __restrict__ S, const int2* __restrict__ work) {
  const int2 w = work[blockIdx.x];
  const SolveDev& s = S[w.x];
  const FM_GLOBAL Ctrl* C = gconst(s.ctrl);
  if (C->status != ST_RUNNING || !C->aa_pending) return;
  const int k = C->win_n;
  constexpr int SUB = 4, CHUNKS = GRAM_TILE / (256 * SUB);
  const FM_GLOBAL R* slot[MAX_DEPTH];
#pragma unroll
  for (int a = 0; a < MAX_DEPTH; ++a)
    slot[a] = gconst((const R*)s.Dring) + (int64_t)(a < k ? C->win_slot[a] : 0) * 3 * s.Nn;
  double accd[NGRAM];
#pragma unroll
  for (int i = 0; i < NGRAM; ++i) accd[i] = 0;
  for (int ch = 0; ch < CHUNKS; ++ch) {
    const int64_t v0 = (int64_t)w.y * GRAM_TILE + ch * (256 * SUB) + threadIdx.x;
    if (v0 >= s.Nn) break;
    R acc[NGRAM];
#pragma unroll
    for (int i = 0; i < NGRAM; ++i) acc[i] = 0;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      R d[SUB][MAX_DEPTH];
#pragma unroll
      for (int sub = 0; sub < SUB; ++sub) {
        const int64_t v = v0 + sub * 256;
#pragma unroll
        for (int a = 0; a < MAX_DEPTH; ++a) d[sub][a] = (a < k && v < s.Nn) ? slot[a][q * s.Nn + v] : (R)0;
      }
#pragma unroll
      for (int sub = 0; sub < SUB; ++sub) {
        int t = 0;
#pragma unroll
        for (int a = 0; a < MAX_DEPTH; ++a)
#pragma unroll
          for (int b = a; b < MAX_DEPTH; ++b) acc[t++] += d[sub][a] * d[sub][b];
      }
    }
#pragma unroll
    for (int i = 0; i < NGRAM; ++i) accd[i] += (double)acc[i];
  }
  __shared__ double outp[NGRAM];
  block_sum<NGRAM>(accd, outp);
  __syncthreads();
  if (threadIdx.x < NGRAM) gmut(s.part_g)[(int64_t)w.y * NGRAM + threadIdx.x] = outp[threadIdx.x];
}

// One block per solve.
__global__ void __launch_bounds__(256) k_control(const SolveDev* __restrict__ S, const int* __restrict__ ids) {
  const SolveDev& s = S[ids[blockIdx.x]];
  Ctrl* C = s.ctrl;
  if (C->status != ST_RUNNING) return;
  double a[NPART_S] = {0, 0, 0, 0, 0, 0, 0, 0};
  sum_tiles<NPART_S>(s.part_s, s.ntile_s, a);
  __shared__ double tot[8];
  block_sum<8>(a, tot);
  __syncthreads();
  if (threadIdx.x != 0) return;
  const int m = C->m;
  const double sS = tot[0], sD = tot[7];
  double err;
  if (sS > 0) err = s.h * sqrt(sD / sS);
  else err = (sD == 0) ? 0.0 : INFINITY;
  if (!(err == err)) err = INFINITY;
  C->err = err; C->sumD2 = sD; C->sumS2 = sS;
  const double inv_nv = 1.0 / (double)s.Nv;
  double fro = 0;
  for (int i = 0; i < 6; ++i) {
    C->macro[i] = tot[1 + i] * inv_nv;
    fro += (i < 3 ? 1.0 : 2.0) * C->macro[i] * C->macro[i];
  }
  fro = sqrt(fro);
  bool mixed_ok = true;
  double r[6];
  int S_idx[6], ns = 0;
  for (int i = 0; i < 6; ++i)
    if (C->mixed_mask[i]) {
      r[ns] = C->mixed_target[i] - C->macro[i];
      S_idx[ns++] = i;
      if (fabs(r[ns - 1]) > C->tol * fro) mixed_ok = false;
    }
  if (m < C->max_iter + 1) {
    LogEntry& e = s.log[m];
    e.err = err; e.aa = 0;
    for (int i = 0; i < 6; ++i) e.macro[i] = C->macro[i];
    e.stamp = wall_clock64();
    e.rs64 = C->rs64;
    C->log_count = m + 1;
  }
  if (err < C->tol && mixed_ok) { C->status = ST_CONVERGED; return; }
  if (m >= C->max_iter) { C->status = ST_MAXITER; return; }
  // Rounding floor of the FP32 real-space step.  Within 100 tol, an FP32
  // plan whose error falls, over the last RS64_WIN iterations, at less than
  // half its average rate since the start of the increment (or not at all
  // for RS64_STALL iterations) is slowed by the rounding of its FP32 strain,
  // stress and divergence: from the next iterate on the real-space step runs
  // in FP64.  The transforms, the Green operator and the Anderson update
  // only precondition the fixed point, so they stay FP32.  An error that
  // still stalls for STALL_ITERS iterations sits at the floor of the
  // precision; the increment stops there, reported as not converged,
  // instead of running to max_iter.
  bool better = false;
  if (err < 0.99 * C->best_err) {
    C->best_err = err;
    C->best_m = m;
    better = true;
  }
  if (C->fp32 && !C->rs64 && err < 100.0 * C->tol && err > 0) {
    bool slow = !better && m - C->best_m >= RS64_STALL;
    if (m >= 2 * RS64_WIN && m <= C->max_iter) {
      const double e0 = s.log[0].err, ew = s.log[m - RS64_WIN].err;
      if (e0 > err && e0 < INFINITY && ew > 0 && ew < INFINITY)
        slow = slow || log(ew / err) / RS64_WIN < 0.5 * log(e0 / err) / m;
    }
    if (slow) {
      C->rs64 = 1;
      C->best_err = err;
      C->best_m = m;
    }
  } else if (!better && m - C->best_m >= STALL_ITERS && err < 100.0 * C->tol) {
    C->status = ST_MAXITER;
    return;
  }
  if (ns > 0) {
    // Voigt C0 block on the stress-controlled components, solved by Gauss elimination
    double Mx[6][7];
    for (int a2 = 0; a2 < ns; ++a2) {
      for (int b2 = 0; b2 < ns; ++b2) {
        const int ia = S_idx[a2], ib = S_idx[b2];
        double c = 0;
        if (ia < 3 && ib < 3) c = C->lam0 + (ia == ib ? 2.0 * C->mu0 : 0.0);
        else if (ia == ib) c = 2.0 * C->mu0;
        Mx[a2][b2] = c;
      }
      Mx[a2][ns] = r[a2];
    }
    for (int p = 0; p < ns; ++p) {
      int piv = p;
      for (int q = p + 1; q < ns; ++q) if (fabs(Mx[q][p]) > fabs(Mx[piv][p])) piv = q;
      for (int c = 0; c <= ns; ++c) { double t = Mx[p][c]; Mx[p][c] = Mx[piv][c]; Mx[piv][c] = t; }
      for (int q = p + 1; q < ns; ++q) {
        const double f = Mx[q][p] / Mx[p][p];
        for (int c = p; c <= ns; ++c) Mx[q][c] -= f * Mx[p][c];
      }
    }
    double dE[6];
    for (int p = ns - 1; p >= 0; --p) {
      double t = Mx[p][ns];
      for (int c = p + 1; c < ns; ++c) t -= Mx[p][c] * dE[c];
      dE[p] = t / Mx[p][p];
    }
    const int vi[6] = {0, 1, 2, 1, 0, 0}, vj[6] = {0, 1, 2, 2, 2, 1};
    for (int p = 0; p < ns; ++p) {
      const int i = vi[S_idx[p]], j = vj[S_idx[p]];
      if (i == j) C->G[i * 3 + i] += dE[p];
      else { C->G[i * 3 + j] += dE[p]; C->G[j * 3 + i] += dE[p]; }
    }
    for (int i = 0; i < 9; ++i) C->g32[i] = (float)C->G[i];
  }
  const int depth = C->depth;
  const int wn = min(depth, m + 1);
  C->win_n = wn;
  for (int j = 0; j < MAX_DEPTH; ++j) C->win_slot[j] = j < wn ? (m - wn + 1 + j) % depth : 0;
  C->n_d = 1; C->slot_d[0] = m % depth; C->alpha[0] = 1.0;
  C->n_b = 0;
  C->slot_w = m % depth;
  C->aa_applied = 0;
  C->aa_pending = (depth > 1 && m >= 2 && (m % C->period) == 0 && wn >= 2) ? 1 : 0;
}

__global__ void __launch_bounds__(256) k_alpha(const SolveDev* __restrict__ S, const int* __restrict__ ids) {
  const SolveDev& s = S[ids[blockIdx.x]];
  Ctrl* C = s.ctrl;
  if (C->status != ST_RUNNING) return;
  if (C->aa_pending) {
    double a[NGRAM];
#pragma unroll
    for (int i = 0; i < NGRAM; ++i) a[i] = 0;
    sum_tiles<NGRAM>(s.part_g, s.ntile_d, a);
    __shared__ double g[NGRAM];
    block_sum<NGRAM>(a, g);
    __syncthreads();
    if (threadIdx.x != 0) return;
    const int k = C->win_n;
    double F[MAX_DEPTH][MAX_DEPTH];
    int t = 0;
    for (int i = 0; i < MAX_DEPTH; ++i)
      for (int j = i; j < MAX_DEPTH; ++j) { F[i][j] = g[t]; F[j][i] = g[t]; ++t; }
    double tr = 0;
    for (int i = 0; i < k; ++i) tr += F[i][i];
    for (int i = 0; i < k; ++i) F[i][i] += 1e-14 * tr;
    // Cholesky; skip the acceleration if a pivot collapses
    double Lc[MAX_DEPTH][MAX_DEPTH] = {};
    bool ok = tr > 0;
    double dmin = INFINITY, dmax = 0;
    for (int j = 0; j < k && ok; ++j) {
      double sdiag = F[j][j];
      for (int p = 0; p < j; ++p) sdiag -= Lc[j][p] * Lc[j][p];
      if (!(sdiag > 0)) { ok = false; break; }
      Lc[j][j] = sqrt(sdiag);
      dmin = fmin(dmin, sdiag); dmax = fmax(dmax, sdiag);
      for (int i = j + 1; i < k; ++i) {
        double sv = F[i][j];
        for (int p = 0; p < j; ++p) sv -= Lc[i][p] * Lc[j][p];
        Lc[i][j] = sv / Lc[j][j];
      }
    }
    if (ok && dmin <= 1e-12 * dmax) ok = false;
    if (ok) {
      double y[MAX_DEPTH];
      for (int i = 0; i < k; ++i) {
        double sv = 1.0;
        for (int p = 0; p < i; ++p) sv -= Lc[i][p] * y[p];
        y[i] = sv / Lc[i][i];
      }
      for (int i = k - 1; i >= 0; --i) {
        double sv = y[i];
        for (int p = i + 1; p < k; ++p) sv -= Lc[p][i] * y[p];
        y[i] = sv / Lc[i][i];
      }
      double sy = 0;
      for (int i = 0; i < k; ++i) sy += y[i];
      if (sy != 0 && sy == sy) {
        C->n_d = k;
        double cum = 0;
        for (int i = 0; i < k; ++i) {
          C->alpha[i] = y[i] / sy;
          C->slot_d[i] = C->win_slot[i];
        }
        const int lo = C->m - k + 1;
        C->n_b = k - 1;
        for (int i = 0; i < k - 1; ++i) {
          cum += C->alpha[i];
          C->beta[i] = cum;
          C->slot_b[i] = (lo + i) % C->depth;
        }
        C->aa_applied = 1;
        if (C->m < C->max_iter + 1) s.log[C->m].aa = 1;
      }
    }
    C->aa_pending = 0;
    C->m += 1;
  } else if (threadIdx.x == 0) {
    C->m += 1;
  }
}

// u = u^f + u* at the nodes (FP64 output).
__global__ void __launch_bounds__(256) k_out_u(const SolveDev* __restrict__ S, int sid) {
  const SolveDev& s = S[sid];
  const Ctrl* C = s.ctrl;
  const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (v >= s.Nn || !s.out_u) return;
  const int N0 = s.N[0], N1 = s.N[1];
  const double X[3] = {(double)(v % N0) * s.h, (double)((v / N0) % N1) * s.h,
                       (double)(v / ((int64_t)N0 * N1)) * s.h};
  for (int q = 0; q < 3; ++q) {
    double u = C->c[q];
    for (int l = 0; l < 3; ++l) {
      u += C->G[q * 3 + l] * X[l];
      for (int m = 0; m < 3; ++m) u += 0.5 * C->H[(q * 3 + l) * 3 + m] * X[l] * X[m];
    }
    s.out_u[q * s.Nn + v] = s.uf[q * s.Nn + v] + u;
  }
}

}  // namespace fm

// Lagrangian finite-strain formulation (Sec. 2.2, Eq. TF_initial and the
// discrete problem of Eq. GeneralBCtobesolved with P in place of sigma):
// F = 1 + grad u at the integration points, first Piola-Kirchhoff stress
// P = F Pi from a hyperelastic law, D = Div P at the nodes with the
// column-wise mirror rules of the small-strain divergence, which hold for a
// non-symmetric tensor as they stand.  The spectral part of an iteration is
// unchanged (B0 / 2mu0 act on the non-symmetric gradient).
//
//  k_fs_stress  one thread per voxel: gradient (FP64, from the FP64
//               displacement), law, S[l][q] = P[q][l] of every point into
//               the solve's stress buffer (9 x n_ppv x voxels, FP64 in both
//               precisions, so that the equilibrium error of an FP32-mixed
//               solve has no FP32 floor).
//  k_fs_div     one block per stress-divergence tile: D_q = sum over the 8
//               voxels J - 1 + b and the directions l of (2 b_l - 1) S_lq of
//               the point owning the corner (HEX1: the point; TETRA2: T1 on
//               odd b, T2 on even b), mirror corners dropped and the sum
//               doubled per reflecting face (reading R21), periodic images
//               along periodic axes of u_q; FP64 partials of sum w |P|^2,
//               <P> (11, 22, 33, 23, 13, 12) and sum |D|^2.
//  k_fs_out     outputs: Green-Lagrange strain and Cauchy stress (Voigt).
#pragma once
#include "fm_space.h"

namespace fm {

// Full displacement gradient g[l][q] = D_l u_q at the points of voxel
// (x, y, z), FP64 (HEX1 weights (2a_l - 1)/(4h); TETRA2 (2a_l - 1)/(2h) on
// the even (T1) and odd (T2) corners), plus the gradient of u*.
__device__ __forceinline__ void voxel_grad64(const SolveDev& s, const FM_GLOBAL Ctrl* C, int x, int y, int z,
                                             double g[2][3][3]) {
  double u[3][8], gA[3][3], gB[3][3], hc[3][3];
  voxel_corners<double>(s, x, y, z, u);
  ustar_grad_column<double>(s, C, x, y, gA, gB);
  tet_cross_terms<double>(s, C, hc);
  const double zc = (z + 0.5) * s.h;
  const int np = s.scheme == 1 ? 2 : 1;
  const double f = s.scheme == 1 ? 0.5 / s.h : 0.25 / s.h;
  for (int r = 0; r < np; ++r)
    for (int l = 0; l < 3; ++l)
      for (int q = 0; q < 3; ++q) {
        double a = 0;
        for (int c = 0; c < 8; ++c) {
          const int bit[3] = {c & 1, (c >> 1) & 1, c >> 2};
          if (s.scheme == 1 && ((bit[0] + bit[1] + bit[2]) & 1) != r) continue;
          a += bit[l] ? u[q][c] : -u[q][c];
        }
        double v = a * f + gA[l][q] + gB[l][q] * zc;
        if (s.scheme == 1) v += r == 0 ? -hc[l][q] : hc[l][q];
        g[r][l][q] = v;
      }
}

__device__ __forceinline__ double det3(const double F[3][3]) {
  return F[0][0] * (F[1][1] * F[2][2] - F[1][2] * F[2][1]) - F[0][1] * (F[1][0] * F[2][2] - F[1][2] * F[2][0]) +
         F[0][2] * (F[1][0] * F[2][1] - F[1][1] * F[2][0]);
}

// First Piola-Kirchhoff stress P[q][J] for F[q][J]: Saint Venant-Kirchhoff
// Pi = lambda tr(E) 1 + 2 mu E, P = F Pi (table entry: lambda, mu);
// compressible Neo-Hookean of Appendix B, P = mu J^-2/3 (F - tr(F F^T)/3
// F^-T) + K (J - 1) J F^-T (table entry: mu, K).
template <typename PT>
__device__ __forceinline__ void pk1_law(int law, PT M, const double F[3][3], double P[3][3]) {
  if (law == LAW_SVK) {
    const double lam = (double)M[0], mu = (double)M[1];
    double E[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double a = 0;
        for (int k = 0; k < 3; ++k) a += F[k][i] * F[k][j];
        E[i][j] = 0.5 * (a - (i == j ? 1.0 : 0.0));
      }
    const double tr = E[0][0] + E[1][1] + E[2][2];
    double Pi[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) Pi[i][j] = 2.0 * mu * E[i][j] + (i == j ? lam * tr : 0.0);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double a = 0;
        for (int k = 0; k < 3; ++k) a += F[i][k] * Pi[k][j];
        P[i][j] = a;
      }
  } else {
    const double mu = (double)M[0], K = (double)M[1];
    const double J = det3(F);
    // F^-T = cof(F) / J
    double cof[3][3];
    cof[0][0] = F[1][1] * F[2][2] - F[1][2] * F[2][1];
    cof[0][1] = F[1][2] * F[2][0] - F[1][0] * F[2][2];
    cof[0][2] = F[1][0] * F[2][1] - F[1][1] * F[2][0];
    cof[1][0] = F[0][2] * F[2][1] - F[0][1] * F[2][2];
    cof[1][1] = F[0][0] * F[2][2] - F[0][2] * F[2][0];
    cof[1][2] = F[0][1] * F[2][0] - F[0][0] * F[2][1];
    cof[2][0] = F[0][1] * F[1][2] - F[0][2] * F[1][1];
    cof[2][1] = F[0][2] * F[1][0] - F[0][0] * F[1][2];
    cof[2][2] = F[0][0] * F[1][1] - F[0][1] * F[1][0];
    double I1 = 0;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) I1 += F[i][j] * F[i][j];
    const double a = mu * pow(J, -2.0 / 3.0), b = K * (J - 1.0) * J;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        const double fit = cof[i][j] / J;
        P[i][j] = a * (F[i][j] - I1 / 3.0 * fit) + b * fit;
      }
  }
}

template <typename R>
__global__ void __launch_bounds__(256) k_fs_stress(const SolveDev* __restrict__ S, const int2* __restrict__ work) {
  const int2 w = work[blockIdx.x / (SPACE_TILE / 256)];
  const SolveDev& s = S[w.x];
  const FM_GLOBAL Ctrl* C = gconst(s.ctrl);
  if (C->status != ST_RUNNING) return;
  const int64_t v = (int64_t)w.y * SPACE_TILE + (blockIdx.x % (SPACE_TILE / 256)) * 256 + threadIdx.x;
  if (v >= s.Nv) return;
  const int n0 = s.n[0], n1 = s.n[1];
  const int x = (int)(v % n0);
  const int64_t t = v / n0;
  const int y = (int)(t % n1), z = (int)(t / n1);
  double g[2][3][3];
  voxel_grad64(s, C, x, y, z, g);
  const int mt = gconst(s.mat)[v];
  const int law = gconst(s.mlaw)[mt];
  const FM_GLOBAL R* M = gconst((const R*)s.mtab) + (int64_t)mt * MT_STRIDE;
  for (int r = 0; r < s.nppv; ++r) {
    double F[3][3], P[3][3];
    for (int q = 0; q < 3; ++q)
      for (int J = 0; J < 3; ++J) F[q][J] = (q == J ? 1.0 : 0.0) + g[r][J][q];
    pk1_law(law, M, F, P);
    for (int l = 0; l < 3; ++l)
      for (int q = 0; q < 3; ++q)
        gmut((double*)s.sig)[((int64_t)(l * 3 + q) * s.nppv + r) * s.Nv + v] = P[q][l];
  }
}

// Divergence of S at the nodes of one stress-divergence tile.
template <typename R>
__global__ void __launch_bounds__(256) k_fs_div(const SolveDev* __restrict__ S, const int2* __restrict__ work) {
  const int2 w = work[blockIdx.x];
  const SolveDev& s = S[w.x];
  const FM_GLOBAL Ctrl* C = gconst(s.ctrl);
  if (C->status != ST_RUNNING) return;
  const SdBox bx = sd_box(s, w.y);
  const int X0 = bx.X0, Y0 = bx.Y0, Z0 = bx.Z0;
  const int X1 = min(X0 + bx.W - 1, s.N[0]), Y1 = min(Y0 + bx.H - 1, s.N[1]), Z1 = min(Z0 + s.sd_zc, s.N[2]);
  const int nx = X1 - X0, ny = Y1 - Y0, nz = Z1 - Z0;
  const int n[3] = {s.n[0], s.n[1], s.n[2]};
  const FM_GLOBAL double* Sg = gconst((const double*)s.sig);
  FM_GLOBAL R* Dring = gmut((R*)s.Dring) + (int64_t)(C->m % s.depth) * 3 * s.Nn;
  const double wip = 1.0 / s.nppv;
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int idx = threadIdx.x; idx < nx * ny * nz; idx += blockDim.x) {
    const int J[3] = {X0 + idx % nx, Y0 + (idx / nx) % ny, Z0 + idx / (nx * ny)};
    const int64_t node = ((int64_t)J[2] * s.N[1] + J[1]) * s.N[0] + J[0];
    for (int q = 0; q < 3; ++q) {
      bool kept = true;
      double fac = 0.25 / s.h;
      for (int i = 0; i < 3; ++i) {
        kept = kept && node_kept(s.kinds[q][i], n[i], J[i]);
        if (s.kinds[q][i] != K_DFT && (J[i] == 0 || J[i] == n[i])) fac *= 2.0;
      }
      double D = 0;
      if (kept) {
        for (int b = 0; b < 8; ++b) {
          const int bb[3] = {b & 1, (b >> 1) & 1, b >> 2};
          int vi[3];
          bool in = true;
          for (int i = 0; i < 3; ++i) {
            int v = J[i] - 1 + bb[i];
            if (v < 0 || v >= n[i]) {
              if (s.kinds[q][i] == K_DFT) v = (v + n[i]) % n[i];
              else in = false;    // mirror corner: dropped, the sum is doubled per reflecting face
            }
            vi[i] = v;
          }
          if (!in) continue;
          const int r = s.nppv == 2 ? (((bb[0] + bb[1] + bb[2]) & 1) ? 0 : 1) : 0;
          const int64_t vox = ((int64_t)vi[2] * n[1] + vi[1]) * n[0] + vi[0];
          for (int l = 0; l < 3; ++l) {
            const double v = Sg[((int64_t)(l * 3 + q) * s.nppv + r) * s.Nv + vox];
            D += bb[l] ? v : -v;
          }
        }
        D *= fac;
        if (C->has_trac) D += node_dstar<double>(s, C, J[0], J[1], J[2], q);
      }
      Dring[q * s.Nn + node] = (R)D;
      acc[7] += D * D;
    }
    // the voxel whose lower corner is this node enters the stress partials once
    if (J[0] < n[0] && J[1] < n[1] && J[2] < n[2]) {
      const int64_t vox = ((int64_t)J[2] * n[1] + J[1]) * n[0] + J[0];
      for (int r = 0; r < s.nppv; ++r) {
        double Sv[3][3];
        for (int l = 0; l < 3; ++l)
          for (int q = 0; q < 3; ++q) Sv[l][q] = Sg[((int64_t)(l * 3 + q) * s.nppv + r) * s.Nv + vox];
        double f2 = 0;
        for (int l = 0; l < 3; ++l)
          for (int q = 0; q < 3; ++q) f2 += Sv[l][q] * Sv[l][q];
        acc[0] += wip * f2;
        // <P> entries P_11, P_22, P_33, P_23, P_13, P_12 (S[l][q] = P[q][l])
        acc[1] += wip * Sv[0][0];
        acc[2] += wip * Sv[1][1];
        acc[3] += wip * Sv[2][2];
        acc[4] += wip * Sv[2][1];
        acc[5] += wip * Sv[2][0];
        acc[6] += wip * Sv[1][0];
      }
    }
  }
  __shared__ double outp[8];
  block_sum<8>(acc, outp);
  __syncthreads();
  if (threadIdx.x < 8) gmut(s.part_s)[(int64_t)w.y * NPART_S + threadIdx.x] = outp[threadIdx.x];
}

// Outputs of a finite-strain solve: Green-Lagrange strain E and Cauchy
// stress J^-1 P F^T at every point (Voigt xx yy zz yz xz xy, FP64).
template <typename R>
__global__ void __launch_bounds__(256) k_fs_out(const SolveDev* __restrict__ S, const int2* __restrict__ work) {
  const int2 w = work[blockIdx.x];
  const SolveDev& s = S[w.x];
  const FM_GLOBAL Ctrl* C = gconst(s.ctrl);
  for (int sub = 0; sub < SPACE_TILE / 256; ++sub) {
    const int64_t v = (int64_t)w.y * SPACE_TILE + sub * 256 + threadIdx.x;
    if (v >= s.Nv) continue;
    const int n0 = s.n[0], n1 = s.n[1];
    const int x = (int)(v % n0);
    const int64_t t = v / n0;
    const int y = (int)(t % n1), z = (int)(t / n1);
    double g[2][3][3];
    voxel_grad64(s, C, x, y, z, g);
    const int mt = gconst(s.mat)[v];
    const int law = gconst(s.mlaw)[mt];
    const FM_GLOBAL R* M = gconst((const R*)s.mtab) + (int64_t)mt * MT_STRIDE;
    const int vi[6] = {0, 1, 2, 1, 0, 0}, vj[6] = {0, 1, 2, 2, 2, 1};
    for (int r = 0; r < s.nppv; ++r) {
      double F[3][3], P[3][3];
      for (int q = 0; q < 3; ++q)
        for (int J = 0; J < 3; ++J) F[q][J] = (q == J ? 1.0 : 0.0) + g[r][J][q];
      pk1_law(law, M, F, P);
      const double J = det3(F);
      for (int k = 0; k < 6; ++k) {
        const int i = vi[k], j = vj[k];
        double e = 0, sg = 0;
        for (int a = 0; a < 3; ++a) {
          e += F[a][i] * F[a][j];
          sg += P[i][a] * F[j][a];
        }
        if (s.out_eps) gmut(s.out_eps)[((int64_t)k * s.nppv + r) * s.Nv + v] = 0.5 * (e - (i == j ? 1.0 : 0.0));
        if (s.out_sig) gmut(s.out_sig)[((int64_t)k * s.nppv + r) * s.Nv + v] = sg / J;
      }
    }
  }
}

}  // namespace fm

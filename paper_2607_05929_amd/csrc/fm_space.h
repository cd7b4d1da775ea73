// Real-space part of an iteration (Alg. 1, lines 7-10) and the per-solve
// control logic (lines 10-18).
//
//  k_stress  voxel kernel: strain at the integration points from the node
//            displacements (HEX1 Eqs. D1HG-D3HG; TETRA2 Eqs. D1T1T2G-D3T1T2G),
//            plus the discrete gradient of the prescribed field, behaviour
//            law, stress written for the divergence, FP64 block partials of
//            sum_ip w |sigma|^2 and sum sigma (macroscopic stress).
//  k_div     node kernel: D_q = sum_l D_l sigma_lq at the kept nodes, with
//            the stress of the mirror voxels obtained from the symmetry /
//            periodicity of the equation's component (Eq.
//            Continuous_der_symmetry_per on the stress columns; for TETRA2
//            the reflection exchanges the two tetrahedra), FP64 partial of
//            sum |D|^2.
//  k_gram    Gram matrix of the residual history (Anderson, FP64 partials).
//  k_control convergence test (Eq. equilibrium_condition), macroscopic
//            stress, mixed loading update, Anderson schedule.
//  k_alpha   Anderson least squares (FP64 normal equations, Cholesky).
#pragma once
#include "fm_laws.h"

namespace fm {

constexpr int SPACE_TILE = 1024;   // voxels / nodes per 256-thread block (4 per thread)

__device__ __forceinline__ int vidx(int l, int q) {
  // Voigt index of the symmetric pair (l, q): xx yy zz yz xz xy
  return l == q ? l : 6 - l - q;
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

// Extension of u_q at the low / high face of an axis: 1 symmetric, -1
// anti-symmetric, 0 periodic.
__device__ __forceinline__ int face_ext(int kind, int side) {
  switch (kind) {
    case K_DFT: return 0;
    case K_DCT1: return 1;
    case K_DST1: return -1;
    case K_DCT3: return side == 0 ? 1 : -1;
    default: return side == 0 ? -1 : 1;
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

// mode 0: iteration; mode 1: commit (state update + FP64 outputs).
// PL = 0 compiles the elastic laws only (no internal variables), PL = 1 all laws.
template <typename R, int PL>
__global__ void __launch_bounds__(256) k_stress(const SolveDev* __restrict__ S, const int2* __restrict__ work, int mode) {
  const int2 w = work[blockIdx.x];
  const SolveDev& s = S[w.x];
  const Ctrl* C = s.ctrl;
  if (mode == 0 && C->status != ST_RUNNING) return;
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int sub = 0; sub < SPACE_TILE / 256; ++sub) {
  const int64_t v = (int64_t)w.y * SPACE_TILE + sub * 256 + threadIdx.x;
  if (v < s.Nv) {
    const int n0 = s.n[0], n1 = s.n[1];
    const int x = (int)(v % n0);
    const int64_t t = v / n0;
    const int y = (int)(t % n1), z = (int)(t / n1);
    const int64_t N0 = s.N[0], N01 = (int64_t)s.N[0] * s.N[1];
    const int64_t base = z * N01 + (int64_t)y * N0 + x;
    double u[3][8];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const double* uq = s.uf + q * s.Nn;
#pragma unroll
      for (int cidx = 0; cidx < 8; ++cidx) {
        const int a = cidx & 1, b = (cidx >> 1) & 1, c = cidx >> 2;
        u[q][cidx] = uq[base + a + b * N0 + c * N01];
      }
    }
    const double h = s.h;
    const double xc[3] = {(x + 0.5) * h, (y + 0.5) * h, (z + 0.5) * h};
    // gradient of u* at the voxel centre
    double gs[3][3];
#pragma unroll
    for (int l = 0; l < 3; ++l)
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        double g = C->G[q * 3 + l];
#pragma unroll
        for (int m = 0; m < 3; ++m) g += C->H[(q * 3 + l) * 3 + m] * xc[m];
        gs[l][q] = g;
      }
    const int mt = s.mat[v];
    const int law = s.mlaw[mt];
    const R* P = (const R*)s.mtab + (int64_t)mt * MT_STRIDE;
    const double wip = 1.0 / s.nppv;
    for (int r = 0; r < s.nppv; ++r) {
      double g[3][3];
      const double f = (s.scheme == 0) ? 0.25 / h : 0.5 / h;
#pragma unroll
      for (int l = 0; l < 3; ++l)
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          double a = 0;
#pragma unroll
          for (int cidx = 0; cidx < 8; ++cidx) {
            const int bit[3] = {cidx & 1, (cidx >> 1) & 1, cidx >> 2};
            const int par = (bit[0] + bit[1] + bit[2]) & 1;
            // HEX1: all corners; TETRA2: T1 = even corners, T2 = odd corners
            if (s.scheme == 1 && par != r) continue;
            a += bit[l] ? u[q][cidx] : -u[q][cidx];
          }
          g[l][q] = a * f + gs[l][q];
        }
      if (s.scheme == 1) {
        // discrete gradient of the cross terms x_a x_b of u* on one tetrahedron
        const double corr = (r == 0 ? -0.5 : 0.5) * h;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          g[0][q] += corr * C->H[(q * 3 + 1) * 3 + 2];
          g[1][q] += corr * C->H[(q * 3 + 0) * 3 + 2];
          g[2][q] += corr * C->H[(q * 3 + 0) * 3 + 1];
        }
      }
      R eps[6] = {(R)g[0][0], (R)g[1][1], (R)g[2][2], (R)(0.5 * (g[1][2] + g[2][1])),
                  (R)(0.5 * (g[0][2] + g[2][0])), (R)(0.5 * (g[0][1] + g[1][0]))};
      R st[7], stn[7];
      R* state = (R*)s.state;
      if (PL && s.has_state) {
#pragma unroll
        for (int k = 0; k < 7; ++k) st[k] = state[((int64_t)k * s.nppv + r) * s.Nv + v];
      } else {
#pragma unroll
        for (int k = 0; k < 7; ++k) st[k] = 0;
      }
      R sig[6];
      if (PL) law_eval<R>(law, P, eps, sig, st, stn, (R)C->dt);
      else law_elastic<R>(law, P, eps, sig, st, stn);
      if (mode == 0) {
        R* so = (R*)s.sig;
#pragma unroll
        for (int k = 0; k < 6; ++k) so[((int64_t)k * s.nppv + r) * s.Nv + v] = sig[k];
        double n2 = 0;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          const double sk = sig[k];
          n2 += (k < 3 ? 1.0 : 2.0) * sk * sk;
          acc[1 + k] += wip * sk;
        }
        acc[0] += wip * n2;
      } else {
        if (PL && s.has_state && (law == LAW_J2 || law == LAW_CP)) {
#pragma unroll
          for (int k = 0; k < 7; ++k) state[((int64_t)k * s.nppv + r) * s.Nv + v] = stn[k];
        }
        if (s.out_eps) {
#pragma unroll
          for (int k = 0; k < 6; ++k) s.out_eps[((int64_t)k * s.nppv + r) * s.Nv + v] = (double)eps[k];
        }
        if (s.out_sig) {
#pragma unroll
          for (int k = 0; k < 6; ++k) s.out_sig[((int64_t)k * s.nppv + r) * s.Nv + v] = (double)sig[k];
        }
      }
    }
  }
  }
  if (mode == 0) {
    __shared__ double outp[7];
    block_sum<7>(acc, outp);
    __syncthreads();
    if (threadIdx.x < 7) s.part_s[(int64_t)w.y * NPART_S + threadIdx.x] = outp[threadIdx.x];
  }
}

template <typename R>
__global__ void __launch_bounds__(256) k_div(const SolveDev* __restrict__ S, const int2* __restrict__ work) {
  const int2 w = work[blockIdx.x];
  const SolveDev& s = S[w.x];
  const Ctrl* C = s.ctrl;
  if (C->status != ST_RUNNING) return;
  double acc[1] = {0};
  for (int sub = 0; sub < SPACE_TILE / 256; ++sub) {
  const int64_t v = (int64_t)w.y * SPACE_TILE + sub * 256 + threadIdx.x;
  if (v < s.Nn) {
    const int N0 = s.N[0], N1 = s.N[1];
    const int J[3] = {(int)(v % N0), (int)((v / N0) % N1), (int)(v / ((int64_t)N0 * N1))};
    const R* sg = (const R*)s.sig;
    R* Dout = (R*)s.Dring + (int64_t)(C->m % s.depth) * 3 * s.Nn;
    const R f = (R)(0.25 / s.h);
    for (int q = 0; q < 3; ++q) {
      bool kept = true;
#pragma unroll
      for (int i = 0; i < 3; ++i) kept = kept && node_kept(s.kinds[q][i], s.n[i], J[i]);
      R D = 0;
      if (kept) {
        for (int cidx = 0; cidx < 8; ++cidx) {
          const int bit[3] = {cidx & 1, (cidx >> 1) & 1, cidx >> 2};
          int vi[3];
          int nref = 0;
          R sgn[3] = {1, 1, 1};
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            int idx = J[i] - 1 + bit[i];
            if (idx < 0 || idx >= s.n[i]) {
              const int side = idx < 0 ? 0 : 1;
              const int e = face_ext(s.kinds[q][i], side);
              if (e == 0) {
                idx = idx < 0 ? s.n[i] - 1 : 0;
              } else {
                idx = idx < 0 ? 0 : s.n[i] - 1;
                ++nref;
#pragma unroll
                for (int l = 0; l < 3; ++l) {
                  // symmetric u_q: + for l != i; anti-symmetric: + for l == i
                  const bool plus = (e == 1) ? (l != i) : (l == i);
                  if (!plus) sgn[l] = -sgn[l];
                }
              }
            }
            vi[i] = idx;
          }
          int r = 0;
          if (s.scheme == 1) {
            const int par = (bit[0] + bit[1] + bit[2]) & 1;
            r = par ? 0 : 1;            // odd corners take T1 values, even corners T2
            if (nref & 1) r ^= 1;       // a reflection exchanges T1 and T2
          }
          const int64_t vox = ((int64_t)vi[2] * s.n[1] + vi[1]) * s.n[0] + vi[0];
#pragma unroll
          for (int l = 0; l < 3; ++l) {
            const R val = sg[((int64_t)vidx(l, q) * s.nppv + r) * s.Nv + vox] * sgn[l];
            D += bit[l] ? val : -val;
          }
        }
        D *= f;
        acc[0] += (double)D * (double)D;
      }
      Dout[q * s.Nn + v] = D;
    }
  }
  }
  __shared__ double outp[1];
  block_sum<1>(acc, outp);
  __syncthreads();
  if (threadIdx.x == 0) s.part_d[w.y] = outp[0];
}

template <typename R>
__global__ void __launch_bounds__(256) k_gram(const SolveDev* __restrict__ S, const int2* __restrict__ work) {
  const int2 w = work[blockIdx.x];
  const SolveDev& s = S[w.x];
  const Ctrl* C = s.ctrl;
  if (C->status != ST_RUNNING || !C->aa_pending) return;
  double acc[NGRAM];
#pragma unroll
  for (int i = 0; i < NGRAM; ++i) acc[i] = 0;
  const int k = C->win_n;
  for (int sub = 0; sub < SPACE_TILE / 256; ++sub) {
  const int64_t v = (int64_t)w.y * SPACE_TILE + sub * 256 + threadIdx.x;
  if (v < s.Nn) {
    const int N0 = s.N[0], N1 = s.N[1];
    const int J[3] = {(int)(v % N0), (int)((v / N0) % N1), (int)(v / ((int64_t)N0 * N1))};
    const R* ring = (const R*)s.Dring;
    for (int q = 0; q < 3; ++q) {
      bool kept = true;
#pragma unroll
      for (int i = 0; i < 3; ++i) kept = kept && node_kept(s.kinds[q][i], s.n[i], J[i]);
      if (!kept) continue;
      double d[MAX_DEPTH];
#pragma unroll
      for (int a = 0; a < MAX_DEPTH; ++a)
        d[a] = a < k ? (double)ring[((int64_t)C->win_slot[a] * 3 + q) * s.Nn + v] : 0.0;
      int t = 0;
#pragma unroll
      for (int a = 0; a < MAX_DEPTH; ++a)
#pragma unroll
        for (int b = a; b < MAX_DEPTH; ++b) acc[t++] += d[a] * d[b];
    }
  }
  }
  __shared__ double outp[NGRAM];
  block_sum<NGRAM>(acc, outp);
  __syncthreads();
  if (threadIdx.x < NGRAM) s.part_g[(int64_t)w.y * NGRAM + threadIdx.x] = outp[threadIdx.x];
}

// One block per solve.
__global__ void __launch_bounds__(256) k_control(const SolveDev* __restrict__ S, const int* __restrict__ ids) {
  const SolveDev& s = S[ids[blockIdx.x]];
  Ctrl* C = s.ctrl;
  if (C->status != ST_RUNNING) return;
  double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int t = threadIdx.x; t < s.ntile_s; t += blockDim.x)
#pragma unroll
    for (int i = 0; i < 7; ++i) a[i] += s.part_s[(int64_t)t * NPART_S + i];
  for (int t = threadIdx.x; t < s.ntile_d; t += blockDim.x) a[7] += s.part_d[t];
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
    C->log_count = m + 1;
  }
  if (err < C->tol && mixed_ok) { C->status = ST_CONVERGED; return; }
  if (m >= C->max_iter) { C->status = ST_MAXITER; return; }
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
    for (int t = threadIdx.x; t < s.ntile_d; t += blockDim.x)
#pragma unroll
      for (int i = 0; i < NGRAM; ++i) a[i] += s.part_g[(int64_t)t * NGRAM + i];
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

// Axis passes of the 3D discrete transforms (Sec. 2.4, Sec. 2.7.2 "Domain
// decomposition and discrete transformations"), one kernel launch per pass
// covering every (solve, component) of a batch through a work list.
//
// One kernel template serves all passes:
//   XP = 1: x pencils (rows contiguous in memory; a block takes 2F or F rows)
//   XP = 0: y or z pencils (a block takes consecutive x positions, so every
//           row of the tile is one contiguous 128-byte segment)
//   MODE 0: forward; MODE 1: inverse; MODE 2: forward, Green operator,
//           inverse (the z pass; the spectrum never leaves LDS).
// The x forward pass reads the Anderson combination sum_j alpha_j D_j of the
// residual ring; the x inverse pass ends with the displacement update.
//
// Each pencil's transform is a complex FFT of length L = S_f n of the
// virtually extended field, built by scattering the node values into LDS.
// Two real pencils travel as the real and imaginary part of one complex
// pencil: the trigonometric transforms have real matrices, so the packed
// result is G_a + i G_b directly; only the periodic r2c / c2r step needs the
// conjugate-symmetry separation.  The FFT runs in place in one LDS buffer,
// each Stockham stage staged through registers (read all, barrier, write).
#pragma once
#include "fm_fft.h"

namespace fm {

constexpr int PASS_THREADS = 1024;
constexpr int PASS_MAXPTS = 7680;      // F * L bound for register staging

// LDS position of element e of a pencil (identity; a padded layout costs
// more registers than its bank-conflict savings in this kernel).
__device__ __forceinline__ int PD(int e) { return e; }
__host__ __device__ inline int pencil_stride(int L) { return L + 4; }

template <typename R>
__device__ __forceinline__ cx<R> ldc(const void* base, int64_t idx) {
  const R* p = (const R*)base + 2 * idx;
  return mk<R>(p[0], p[1]);
}
template <typename R>
__device__ __forceinline__ void stc(void* base, int64_t idx, cx<R> v) {
  R* p = (R*)base + 2 * idx;
  p[0] = v.re; p[1] = v.im;
}

// ---- in-place Stockham stage, register staged -----------------------------
template <typename R, int RAD>
__device__ __forceinline__ void stage_ip(cx<R>* buf, int F, int L, int LS, int p, const cx<R>* W, bool inv) {
  constexpr int MAXB = (PASS_MAXPTS / RAD + PASS_THREADS - 1) / PASS_THREADS;
  const int T = L / RAD;
  const int tstep = L / (p * RAD);
  const int total = F * T;
  const R sgn = inv ? (R)1 : (R)-1;
  cx<R> u[MAXB][RAD];
#pragma unroll
  for (int kb = 0; kb < MAXB; ++kb) {
    const int b = threadIdx.x + kb * PASS_THREADS;
    if (b < total) {
      const int f = b / T, i = b - f * T;
      const int k = i % p;
      const cx<R>* s = buf + f * LS;
#pragma unroll
      for (int r = 0; r < RAD; ++r) {
        cx<R> v = s[PD(i + r * T)];
        if (r > 0 && k > 0) v = mul(v, twid(W, r * k * tstep, inv));
        u[kb][r] = v;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int kb = 0; kb < MAXB; ++kb) {
    const int b = threadIdx.x + kb * PASS_THREADS;
    if (b < total) {
      const int f = b / T, i = b - f * T;
      const int k = i % p;
      if constexpr (RAD == 2) bfly2(u[kb]);
      else if constexpr (RAD == 3) bfly3(u[kb], sgn);
      else if constexpr (RAD == 4) bfly4(u[kb], sgn);
      else if constexpr (RAD == 5) bfly5(u[kb], sgn);
      else bfly8(u[kb], sgn);
      cx<R>* dd = buf + f * LS;
      const int o0 = (i - k) * RAD + k;
#pragma unroll
      for (int s2 = 0; s2 < RAD; ++s2) dd[PD(o0 + s2 * p)] = u[kb][s2];
    }
  }
  __syncthreads();
}

// Out-of-place stage for radices other than 2, 3, 4, 5, 8 (padded layout).
template <typename R>
__device__ __forceinline__ void stage_gen_pd(const cx<R>* __restrict__ src, cx<R>* __restrict__ dst, int F, int L,
                                             int LS, int p, int RAD, const cx<R>* W, bool inv) {
  const int T = L / RAD;
  const int tstep = L / (p * RAD);
  for (int b = threadIdx.x; b < F * T * RAD; b += blockDim.x) {
    const int s2 = b % RAD;
    const int bb = b / RAD;
    const int f = bb / T, i = bb - f * T;
    const int k = i % p;
    const cx<R>* s = src + f * LS;
    cx<R> acc = mk<R>(0, 0);
    for (int r = 0; r < RAD; ++r) {
      cx<R> v = s[PD(i + r * T)];
      if (r > 0 && k > 0) v = mul(v, twid(W, r * k * tstep, inv));
      const int e = (r * s2) % RAD;
      if (e) v = mul(v, twid(W, e * T, inv));
      acc = add(acc, v);
    }
    dst[f * LS + PD((i - k) * RAD + k + s2 * p)] = acc;
  }
}

// FFT of F pencils in `buf` (stride LS, padded positions).  Radices other
// than 2, 3, 4, 5, 8 go out of place through `aux` (unusual lengths only);
// the returned pointer holds the result.
template <typename R>
__device__ __forceinline__ cx<R>* fft_ip(cx<R>* buf, cx<R>* aux, int F, int L, int LS, int nrad, const int32_t* rad,
                                         const cx<R>* W, bool inv) {
  int p = 1;
  for (int st = 0; st < nrad; ++st) {
    const int RAD = rad[st];
    switch (RAD) {
      case 2: stage_ip<R, 2>(buf, F, L, LS, p, W, inv); break;
      case 3: stage_ip<R, 3>(buf, F, L, LS, p, W, inv); break;
      case 4: stage_ip<R, 4>(buf, F, L, LS, p, W, inv); break;
      case 5: stage_ip<R, 5>(buf, F, L, LS, p, W, inv); break;
      case 8: stage_ip<R, 8>(buf, F, L, LS, p, W, inv); break;
      default: {
        stage_gen_pd<R>(buf, aux, F, L, LS, p, RAD, W, inv);
        __syncthreads();
        cx<R>* t = buf; buf = aux; aux = t;
        break;
      }
    }
    p *= RAD;
  }
  return buf;
}

// ---- extension scatter ----------------------------------------------------
// Node j of a pencil -> positions of the extended field with signs.
__device__ __forceinline__ int ext_targets(int kind, int n, int j, int* pos, int* sg) {
  switch (kind) {
    case K_DFT: pos[0] = j; sg[0] = 1; return 1;
    case K_DCT1:
      pos[0] = j; sg[0] = 1;
      if (j > 0 && j < n) { pos[1] = 2 * n - j; sg[1] = 1; return 2; }
      return 1;
    case K_DST1:
      pos[0] = j; sg[0] = 1; pos[1] = 2 * n - j; sg[1] = -1; return 2;
    case K_DCT3:
      pos[0] = j; sg[0] = 1; pos[1] = 2 * n - j; sg[1] = -1;
      if (j == 0) return 2;
      pos[2] = 2 * n + j; sg[2] = -1; pos[3] = 4 * n - j; sg[3] = 1; return 4;
    default:  // DST3
      pos[0] = j; sg[0] = 1; pos[1] = 4 * n - j; sg[1] = -1;
      if (j == n) return 2;
      pos[2] = 2 * n - j; sg[2] = 1; pos[3] = 2 * n + j; sg[3] = -1; return 4;
  }
}

// Positions of the extended field never written by the node scatter (zeros).
__device__ __forceinline__ int ext_zeros(int kind, int n, int* pos) {
  switch (kind) {
    case K_DST1: pos[0] = 0; pos[1] = n; return 2;
    case K_DCT3: pos[0] = n; pos[1] = 3 * n; return 2;
    case K_DST3: pos[0] = 0; pos[1] = 2 * n; return 2;
    default: return 0;
  }
}

// Coefficient k of the spectrum -> extended-spectrum positions and factors.
template <typename R>
__device__ __forceinline__ int spec_targets(int kind, int n, int k, int* pos, cx<R>* fac) {
  switch (kind) {
    case K_DFT: pos[0] = k; fac[0] = mk<R>(1, 0); return 1;
    case K_DCT1:
      pos[0] = k; fac[0] = mk<R>(1, 0);
      if (k > 0 && k < n) { pos[1] = 2 * n - k; fac[1] = mk<R>(1, 0); return 2; }
      return 1;
    case K_DST1:
      pos[0] = k + 1; fac[0] = mk<R>(0, -1); pos[1] = 2 * n - k - 1; fac[1] = mk<R>(0, 1); return 2;
    case K_DCT3:
      pos[0] = 2 * k + 1; fac[0] = mk<R>(2, 0); pos[1] = 4 * n - 2 * k - 1; fac[1] = mk<R>(2, 0); return 2;
    default:
      pos[0] = 2 * k + 1; fac[0] = mk<R>(0, -2); pos[1] = 4 * n - 2 * k - 1; fac[1] = mk<R>(0, 2); return 2;
  }
}

// Number of zero positions of the extended spectrum and the i-th of them.
__device__ __forceinline__ int spec_nzero(int kind, int n) {
  switch (kind) {
    case K_DST1: return 2;
    case K_DCT3:
    case K_DST3: return 2 * n;
    default: return 0;
  }
}
__device__ __forceinline__ int spec_zero(int kind, int n, int i) {
  if (kind == K_DST1) return i == 0 ? 0 : n;
  return 2 * i;   // even positions of the quarter-wave spectra
}

// ---------------------------------------------------------------------------
// Addressing of a pencil element: column c of the tile, element e along the
// axis.  XP: x rows (element stride 1, column = row); else columns (stride 1
// across columns, element stride sa).
struct Tile {
  int p0b, p1, ncol;
};

template <int XP>
__device__ __forceinline__ int64_t addr(const Tile& t, int c, int e, int64_t sa, int64_t s1) {
  if (XP) return (int64_t)(t.p0b + c) * s1 + e;
  return (int64_t)(t.p0b + c) + (int64_t)e * sa + (int64_t)t.p1 * s1;
}

// Per-column Green data of the fused z pass: den(kz) = A cos^2(xi_z/2) +
// B sin^2(xi_z/2) (the modified-frequency products of Eqs. NSGO2_* are
// linear in the z factors).
template <typename R>
struct GreenCol {
  R A, B;
};

template <typename R>
__device__ __forceinline__ GreenCol<R> green_col(const PassDesc& d, int kx, int ky) {
  GreenCol<R> g;
  const double s0 = d.gs2[0][kx], c0 = d.gc2[0][kx], s1 = d.gs2[1][ky], c1 = d.gc2[1][ky];
  double a[3], b[3];
  if (d.scheme == 0) {
    a[0] = s0 * c1; a[1] = c0 * s1; a[2] = 0;
    b[0] = 0; b[1] = 0; b[2] = c0 * c1;
  } else {
    a[0] = s0 * c1; a[1] = c0 * s1; a[2] = s0 * s1;
    b[0] = c0 * s1; b[1] = s0 * c1; b[2] = c0 * c1;
  }
  const double lam = d.green_lam ? d.lam0 : 0.0;
  const double f = 4.0 / (d.h * d.h);
  g.A = (R)(f * (2.0 * d.mu0 * (a[0] + a[1] + a[2]) + lam * a[d.q]));
  g.B = (R)(f * (2.0 * d.mu0 * (b[0] + b[1] + b[2]) + lam * b[d.q]));
  return g;
}

// 1/x: the hardware reciprocal (1 ulp) in FP32, a correctly rounded
// division in FP64.
template <typename R> __device__ __forceinline__ R recip(R x) { return (R)1 / x; }
template <> __device__ __forceinline__ float recip<float>(float x) { return __builtin_amdgcn_rcpf(x); }

// Green factor 1/den, 0 on the null modes.  The null modes (decided in index
// space: all three frequencies at 0; two or more at pi for HEX1, all three
// for TETRA2) are exactly the zeros of den: the 1D tables hold exact 0 and 1
// at the index-flagged frequencies and values strictly inside (0, 1)
// elsewhere, and den is a sum of non-negative products of them, each term
// vanishing only through a flagged factor.  So den == 0 is the index rule.
template <typename R>
__device__ __forceinline__ R green_apply(const GreenCol<R>& g, R s2, R c2) {
  const R den = g.A * c2 + g.B * s2;
  return den == (R)0 ? (R)0 : recip<R>(den);
}

template <typename R, int MODE, int XP>
__global__ void __launch_bounds__(PASS_THREADS) k_pass(const PassDesc* __restrict__ descs, const int2* __restrict__ work,
                                                       const SolveDev* __restrict__ S) {
  extern __shared__ __align__(16) char smem[];
  __shared__ GreenCol<R> gcol[32];
  const int2 w = work[blockIdx.x];
  const PassDesc& d = descs[w.x];
  const Ctrl* C = S[d.solve].ctrl;
  if (C->status != ST_RUNNING) return;
  const int L = d.L, LS = pencil_stride(L), F = d.F, n = d.n, kind = d.kind;
  cx<R>* buf = (cx<R>*)smem;
  cx<R>* aux = buf + F * LS;       // only sized when a generic radix is present
  const int cols = d.cols;
  Tile t;
  if (XP) { t.p0b = w.y * cols; t.p1 = 0; }
  else { t.p0b = (w.y % d.tiles_p0) * cols; t.p1 = w.y / d.tiles_p0; }
  t.ncol = min(cols, d.n_p0 - t.p0b);
  const bool packed = d.packed;                 // real data, two columns per FFT
  const bool half = packed && kind == K_DFT;    // r2c / c2r along a periodic axis
  const cx<R>* W = (const cx<R>*)d.tw;
  const int nthr = PASS_THREADS;

  if (MODE == 2 && threadIdx.x < cols) {
    const int c = threadIdx.x;
    gcol[c] = green_col<R>(d, min(t.p0b + c, d.n_p0 - 1), t.p1);
  }

  if (MODE == 0 || MODE == 2) {
    // ---- scatter the node values into the extension ----
    int j0, cnt;
    raw_range(kind, n, j0, cnt);
    // Anderson combination (x forward pass)
    const int nd = (XP && MODE == 0) ? C->n_d : 0;
    R al[MAX_DEPTH];
    const R* src[MAX_DEPTH];
    if (XP && MODE == 0) {
#pragma unroll
      for (int q = 0; q < MAX_DEPTH; ++q) {
        al[q] = q < nd ? (R)C->alpha[q] : (R)0;
        src[q] = (const R*)d.ring + (int64_t)(q < nd ? C->slot_d[q] : 0) * d.ring_stride;
      }
    }
    {
      int zp[2];
      const int nz = ext_zeros(kind, n, zp);
      if (nz && threadIdx.x < 2 * F) {
        const int f = threadIdx.x >> 1;
        buf[f * LS + PD((threadIdx.x & 1) ? zp[1] : zp[0])] = mk<R>(0, 0);
      }
    }
    const int nitems = cols * cnt;
    for (int idx = threadIdx.x; idx < nitems; idx += nthr) {
      int c, e;
      if (XP) { c = idx / cnt; e = idx - c * cnt; }
      else { c = idx % cols; e = idx / cols; }
      const int j = j0 + e;
      cx<R> v = mk<R>(0, 0);
      if (c < t.ncol) {
        if (XP && MODE == 0) {
          const int64_t o = addr<1>(t, c, j, 0, d.in_s1);
          R a = al[0] * src[0][o];
#pragma unroll
          for (int q = 1; q < MAX_DEPTH; ++q)
            if (q < nd) a += al[q] * src[q][o];
          v.re = a;
        } else if (d.cplx_in) {
          v = ldc<R>(d.in, addr<XP>(t, c, j, d.in_sa, d.in_s1));
        } else {
          v.re = ((const R*)d.in)[addr<XP>(t, c, j, d.in_sa, d.in_s1)];
        }
      }
      int pos[4], sg[4];
      const int np = ext_targets(kind, n, j, pos, sg);
      if (packed) {
        R* bb = (R*)(buf + (c >> 1) * LS) + (c & 1);
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (k < np) bb[2 * PD(pos[k])] = sg[k] > 0 ? v.re : -v.re;
      } else {
        cx<R>* bb = buf + c * LS;
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (k < np) bb[PD(pos[k])] = sg[k] > 0 ? v : scl(v, (R)-1);
      }
    }
    __syncthreads();
    buf = fft_ip<R>(buf, aux, F, L, LS, d.nrad, d.rad, W, false);
    aux = (buf == (cx<R>*)smem) ? buf + F * LS : (cx<R>*)smem;
  }

  const int M = half ? n / 2 + 1 : n_freq(kind, n);   // coefficients along the axis

  if (MODE == 0) {
    // ---- extract coefficients and store ----
    for (int idx = threadIdx.x; idx < cols * M; idx += nthr) {
      int c, k;
      if (XP) { c = idx / M; k = idx - c * M; }
      else { c = idx % cols; k = idx / cols; }
      if (c >= t.ncol) continue;
      const int64_t o = addr<XP>(t, c, k, d.out_sa, d.out_s1);
      if (half) {
        const cx<R>* Z = buf + (c >> 1) * LS;
        const cx<R> a = Z[PD(k)], b = conj(Z[PD(k == 0 ? 0 : L - k)]);
        const cx<R> v = (c & 1) ? mk<R>((R)0.5 * (a.im - b.im), (R)-0.5 * (a.re - b.re))
                                : scl(add(a, b), (R)0.5);
        stc<R>(d.out, o, v);
      } else {
        int m; R fr, fi;
        coef_src<R>(kind, k, m, fr, fi);
        const cx<R> v = mul((packed ? buf + (c >> 1) * LS : buf + c * LS)[PD(m)], mk<R>(fr, fi));
        if (packed) ((R*)d.out)[o] = (c & 1) ? v.im : v.re;
        else stc<R>(d.out, o, v);
      }
    }
    return;
  }

  if (MODE == 2) {
    // ---- Green operator, in place on the extended spectrum ----
    // Position m holds alpha_m G[k(m)] (Table 1 and the spectrum's parity);
    // scaling G[k] by the factor of its column keeps that structure, so each
    // position is scaled where it lies.  Packed real columns: real alpha
    // scales (re, im) by (f_a, f_b), imaginary alpha by (f_b, f_a).  Periodic
    // r2c columns: positions m and n-m are separated, scaled and recombined.
    const double* zs2 = d.gs2[2];
    const double* zc2 = d.gc2[2];
    if (half) {
      const int npair = n / 2 + 1;
      for (int idx = threadIdx.x; idx < F * npair; idx += nthr) {
        const int f = idx / npair, m = idx - f * npair;
        cx<R>* Z = buf + f * LS;
        const int mm = m == 0 ? 0 : n - m;
        const cx<R> a = Z[PD(m)], b = conj(Z[PD(mm)]);
        const cx<R> A = scl(add(a, b), (R)0.5);
        const cx<R> B = mk<R>((R)0.5 * (a.im - b.im), (R)-0.5 * (a.re - b.re));
        const int c0 = 2 * f, c1 = 2 * f + 1;
        const R s2 = (R)zs2[m], c2 = (R)zc2[m];
        const R fa = (c0 < t.ncol) ? green_apply<R>(gcol[c0], s2, c2) : (R)0;
        const R fb = (c1 < t.ncol) ? green_apply<R>(gcol[c1], s2, c2) : (R)0;
        const cx<R> A2 = scl(A, fa), B2 = scl(B, fb);
        Z[PD(m)] = mk<R>(A2.re - B2.im, A2.im + B2.re);
        if (mm != m) {
          const cx<R> Ac = conj(A2), Bc = conj(B2);
          Z[PD(mm)] = mk<R>(Ac.re - Bc.im, Ac.im + Bc.re);
        }
      }
    } else {
      for (int idx = threadIdx.x; idx < F * L; idx += nthr) {
        const int f = idx / L, m = idx - f * L;
        cx<R>* Z = buf + f * LS;
        int k;
        R fr, fi;
        if (!spec_src<R>(kind, n, m, k, fr, fi)) { Z[PD(m)] = mk<R>(0, 0); continue; }
        const R s2 = (R)zs2[k], c2 = (R)zc2[k];
        if (packed) {
          const int c0 = 2 * f, c1 = 2 * f + 1;
          const R fa = (c0 < t.ncol) ? green_apply<R>(gcol[c0], s2, c2) : (R)0;
          const R fb = (c1 < t.ncol) ? green_apply<R>(gcol[c1], s2, c2) : (R)0;
          const cx<R> z = Z[PD(m)];
          Z[PD(m)] = (fi == (R)0) ? mk<R>(z.re * fa, z.im * fb) : mk<R>(z.re * fb, z.im * fa);
        } else {
          const R g = (f < t.ncol) ? green_apply<R>(gcol[f], s2, c2) : (R)0;
          Z[PD(m)] = scl(Z[PD(m)], g);
        }
      }
    }
    __syncthreads();
  } else {
    // ---- MODE 1: coefficients from memory into the spectral extension ----
    const int Min = d.len_in;
    const int nzs = spec_nzero(kind, n);
    for (int idx = threadIdx.x; idx < F * nzs; idx += nthr)
      buf[(idx / nzs) * LS + PD(spec_zero(kind, n, idx % nzs))] = mk<R>(0, 0);
    if (packed) {
      // two real columns per FFT: v = G_a + i G_b (or the two half spectra)
      for (int idx = threadIdx.x; idx < F * Min; idx += nthr) {
        int f, k;
        if (XP) { f = idx / Min; k = idx - f * Min; }
        else { f = idx % F; k = idx / F; }
        const int c0 = 2 * f, c1 = 2 * f + 1;
        cx<R>* Z = buf + f * LS;
        if (half) {
          cx<R> A = mk<R>(0, 0), B = mk<R>(0, 0);
          if (c0 < t.ncol) A = ldc<R>(d.in, addr<XP>(t, c0, k, d.in_sa, d.in_s1));
          if (c1 < t.ncol) B = ldc<R>(d.in, addr<XP>(t, c1, k, d.in_sa, d.in_s1));
          Z[PD(k)] = mk<R>(A.re - B.im, A.im + B.re);
          if (k > 0 && 2 * k != n) {
            const cx<R> Ac = conj(A), Bc = conj(B);
            Z[PD(n - k)] = mk<R>(Ac.re - Bc.im, Ac.im + Bc.re);
          }
        } else {
          R a = 0, b = 0;
          if (c0 < t.ncol) a = ((const R*)d.in)[addr<XP>(t, c0, k, d.in_sa, d.in_s1)];
          if (c1 < t.ncol) b = ((const R*)d.in)[addr<XP>(t, c1, k, d.in_sa, d.in_s1)];
          const cx<R> v = mk<R>(a, b);
          int pos[2];
          cx<R> fac[2];
          const int np = spec_targets<R>(kind, n, k, pos, fac);
#pragma unroll
          for (int q = 0; q < 2; ++q)
            if (q < np) Z[PD(pos[q])] = mul(v, fac[q]);
        }
      }
    } else {
      for (int idx = threadIdx.x; idx < cols * Min; idx += nthr) {
        int c, k;
        if (XP) { c = idx / Min; k = idx - c * Min; }
        else { c = idx % cols; k = idx / cols; }
        cx<R> v = mk<R>(0, 0);
        if (c < t.ncol) v = ldc<R>(d.in, addr<XP>(t, c, k, d.in_sa, d.in_s1));
        int pos[2];
        cx<R> fac[2];
        const int np = spec_targets<R>(kind, n, k, pos, fac);
        cx<R>* bb = buf + c * LS;
#pragma unroll
        for (int q = 0; q < 2; ++q)
          if (q < np) bb[PD(pos[q])] = mul(v, fac[q]);
      }
    }
    __syncthreads();
  }

  // ---- inverse FFT and node output ----
  buf = fft_ip<R>(buf, aux, F, L, LS, d.nrad, d.rad, W, true);
  const R invL = (R)1 / (R)L;
  const int Nout = n + 1;
  if (XP) {
    // x inverse: displacement update u^f += w - sum_k beta_k delta_k
    const int nb = C->n_b;
    R be[MAX_DEPTH];
    const R* dsrc[MAX_DEPTH];
#pragma unroll
    for (int q = 0; q < MAX_DEPTH; ++q) {
      be[q] = q < nb ? (R)C->beta[q] : (R)0;
      dsrc[q] = (const R*)d.ring + (int64_t)(q < nb ? C->slot_b[q] : 0) * d.ring_stride;
    }
    R* dw = (R*)d.ring + (int64_t)C->slot_w * d.ring_stride;
    for (int idx = threadIdx.x; idx < t.ncol * Nout; idx += nthr) {
      const int r = idx / Nout, j = idx - r * Nout;
      const int x = node_src(kind, n, j);
      R v = 0;
      if (x >= 0) {
        const cx<R> z = buf[(r >> 1) * LS + PD(x)];
        v = ((r & 1) ? z.im : z.re) * invL;
      }
      const int64_t o = (int64_t)(t.p0b + r) * d.out_s1 + j;
      R dl = v;
#pragma unroll
      for (int q = 0; q < MAX_DEPTH; ++q)
        if (q < nb) dl -= be[q] * dsrc[q][o];
      dw[o] = dl;
      d.uf[o] += (double)dl;
    }
    return;
  }
  for (int idx = threadIdx.x; idx < cols * Nout; idx += nthr) {
    const int c = idx % cols, j = idx / cols;
    if (c >= t.ncol) continue;
    const int x = node_src(kind, n, j);
    const int64_t o = addr<0>(t, c, j, d.out_sa, d.out_s1);
    if (packed) {
      R v = 0;
      if (x >= 0) {
        const cx<R> z = buf[(c >> 1) * LS + PD(x)];
        v = ((c & 1) ? z.im : z.re) * invL;
      }
      ((R*)d.out)[o] = v;
    } else {
      cx<R> v = mk<R>(0, 0);
      if (x >= 0) v = scl(buf[c * LS + PD(x)], invL);
      stc<R>(d.out, o, v);
    }
  }
}

}  // namespace fm

// Axis passes of the 3D discrete transforms (Sec. 2.4, Sec. 3.2 "Domain
// decomposition and discrete transformations"), one kernel launch per pass
// covering every (solve, component) of a batch through a work list.
//
//  k_xfwd     x pencils (contiguous rows): Anderson combination of the ring
//             of residual fields, forward DT along x.  Input always real.
//  k_xinv     inverse DT along x, then the displacement update
//             u^f += w - sum_k beta_k delta_k and the new increment delta.
//  k_strided  y or z pencils (columns strided in memory, a block takes
//             consecutive x positions so every row access is contiguous):
//             MODE 0 forward, MODE 1 inverse, MODE 2 forward + Green
//             operator + inverse (the z pass; the spectrum never leaves LDS).
#pragma once
#include "fm_fft.h"

namespace fm {

// Green factor 1/den at spectral indices (k0, k1, k2) of component q:
// den = (4/h^2)(2 mu0 sum_i t_i + lambda0 t_q), Eqs. NSGO2_HEX1 / NSGO2_TETRA2
// with t_i the squared modified-frequency components built from the 1D
// sin^2 / cos^2 tables; 0 on the null modes (decided from index flags).
__device__ __forceinline__ double green_factor(const PassDesc& d, int k0, int k1, int k2) {
  const uint8_t f0 = d.gfl[0][k0], f1 = d.gfl[1][k1], f2 = d.gfl[2][k2];
  const int allz = (f0 & f1 & f2) & 1;
  const int npi = ((f0 >> 1) & 1) + ((f1 >> 1) & 1) + ((f2 >> 1) & 1);
  if (allz) return 0.0;
  if (d.scheme == 0 ? (npi >= 2) : (npi == 3)) return 0.0;
  const double s0 = d.gs2[0][k0], s1 = d.gs2[1][k1], s2 = d.gs2[2][k2];
  const double c0 = d.gc2[0][k0], c1 = d.gc2[1][k1], c2 = d.gc2[2][k2];
  double t0 = s0 * c1 * c2, t1 = c0 * s1 * c2, t2 = c0 * c1 * s2;
  if (d.scheme == 1) { t0 += c0 * s1 * s2; t1 += s0 * c1 * s2; t2 += s0 * s1 * c2; }
  const double tq = d.q == 0 ? t0 : (d.q == 1 ? t1 : t2);
  const double den = (4.0 / (d.h * d.h)) * (2.0 * d.mu0 * (t0 + t1 + t2) + (d.green_lam ? d.lam0 * tq : 0.0));
  return 1.0 / den;
}

// Separate two real sequences packed as Z = Ea + i Eb.
template <typename R>
__device__ __forceinline__ cx<R> unpack(const cx<R>* Z, int L, int m, int which) {
  const cx<R> a = Z[m];
  const cx<R> b = conj(Z[m == 0 ? 0 : L - m]);
  if (which == 0) return scl(add(a, b), (R)0.5);
  const cx<R> d = sub(a, b);                   // -i/2 * d
  return mk<R>((R)0.5 * d.im, (R)-0.5 * d.re);
}

// Coefficient k of the forward transform from the extended spectrum.
template <typename R>
__device__ __forceinline__ cx<R> fwd_coef(const cx<R>* Z, int L, int kind, int k, int packed, int which) {
  int m; R fr, fi;
  coef_src<R>(kind, k, m, fr, fi);
  const cx<R> e = packed ? unpack(Z, L, m, which) : Z[m];
  return mul(e, mk<R>(fr, fi));
}

// Extended spectrum value at position m from coefficients (complex coef
// accessor).  For the r2c-halved DFT axis the Hermitian completion is used.
template <typename R, typename Get>
__device__ __forceinline__ cx<R> spec_value(int kind, int n, int m, bool half, Get get) {
  if (kind == K_DFT) {
    if (half && m > n / 2) return conj(get(n - m));
    return get(m);
  }
  int k; R fr, fi;
  if (!spec_src<R>(kind, n, m, k, fr, fi)) return mk<R>(0, 0);
  return mul(get(k), mk<R>(fr, fi));
}

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

// ---------------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(256) k_xfwd(const PassDesc* __restrict__ descs, const int2* __restrict__ work,
                                              const SolveDev* __restrict__ S) {
  extern __shared__ __align__(16) char smem[];
  const int2 w = work[blockIdx.x];
  const PassDesc& d = descs[w.x];
  const Ctrl* C = S[d.solve].ctrl;
  if (C->status != ST_RUNNING) return;
  const int L = d.L, LS = L + 4, F = d.F, n = d.n, kind = d.kind;
  cx<R>* A = (cx<R>*)smem;
  cx<R>* B = A + F * LS;
  const int rows = d.cols;
  const int row0 = w.y * rows;
  const int nrows = min(rows, d.n_p0 - row0);
  int j0, cnt;
  raw_range(kind, n, j0, cnt);
  const int nd = C->n_d;
  R al[MAX_DEPTH];
  const R* src[MAX_DEPTH];
  for (int t = 0; t < MAX_DEPTH; ++t) {
    al[t] = t < nd ? (R)C->alpha[t] : (R)0;
    src[t] = (const R*)d.ring + (int64_t)(t < nd ? C->slot_d[t] : 0) * d.ring_stride;
  }
  R* raw = (R*)B;
  for (int idx = threadIdx.x; idx < rows * cnt; idx += blockDim.x) {
    const int r = idx / cnt, e = idx - r * cnt;
    R v = 0;
    if (r < nrows) {
      const int64_t off = (int64_t)(row0 + r) * d.in_s1 + (j0 + e);
      v = al[0] * src[0][off];
      for (int t = 1; t < nd; ++t) v += al[t] * src[t][off];
    }
    raw[idx] = v;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < F * L; idx += blockDim.x) {
    const int f = idx / L, x = idx - f * L;
    int j, sg;
    ext_src(kind, n, x, j, sg);
    R a = 0, b = 0;
    if (sg) {
      a = (R)sg * raw[(2 * f) * cnt + (j - j0)];
      b = (R)sg * raw[(2 * f + 1) * cnt + (j - j0)];
    }
    A[f * LS + x] = mk<R>(a, b);
  }
  __syncthreads();
  const cx<R>* Z = lds_fft<R>(A, B, F, L, LS, d.nrad, d.rad, (const cx<R>*)d.tw, false);
  const int M = d.len_out;
  for (int idx = threadIdx.x; idx < nrows * M; idx += blockDim.x) {
    const int r = idx / M, k = idx - r * M;
    const cx<R>* Zf = Z + (r >> 1) * LS;
    const cx<R> v = fwd_coef<R>(Zf, L, kind, k, 1, r & 1);
    const int64_t o = (int64_t)(row0 + r) * d.out_s1 + k;
    if (d.cplx_out) stc<R>(d.out, o, v);
    else ((R*)d.out)[o] = v.re;
  }
}

template <typename R>
__global__ void __launch_bounds__(256) k_xinv(const PassDesc* __restrict__ descs, const int2* __restrict__ work,
                                              const SolveDev* __restrict__ S) {
  extern __shared__ __align__(16) char smem[];
  const int2 w = work[blockIdx.x];
  const PassDesc& d = descs[w.x];
  const Ctrl* C = S[d.solve].ctrl;
  if (C->status != ST_RUNNING) return;
  const int L = d.L, LS = L + 4, F = d.F, n = d.n, kind = d.kind;
  cx<R>* A = (cx<R>*)smem;
  cx<R>* B = A + F * LS;
  const int rows = d.cols;
  const int row0 = w.y * rows;
  const int nrows = min(rows, d.n_p0 - row0);
  const int M = d.len_in;
  // coefficients -> B
  if (d.cplx_in) {
    for (int idx = threadIdx.x; idx < rows * M; idx += blockDim.x) {
      const int r = idx / M, k = idx - r * M;
      B[idx] = r < nrows ? ldc<R>(d.in, (int64_t)(row0 + r) * d.in_s1 + k) : mk<R>(0, 0);
    }
  } else {
    R* raw = (R*)B;
    for (int idx = threadIdx.x; idx < rows * M; idx += blockDim.x) {
      const int r = idx / M, k = idx - r * M;
      raw[idx] = r < nrows ? ((const R*)d.in)[(int64_t)(row0 + r) * d.in_s1 + k] : (R)0;
    }
  }
  __syncthreads();
  const bool half = kind == K_DFT;   // x is always the r2c axis when periodic
  for (int idx = threadIdx.x; idx < F * L; idx += blockDim.x) {
    const int f = idx / L, m = idx - f * L;
    cx<R> za, zb;
    if (d.cplx_in) {
      const cx<R>* ca = B + (2 * f) * M;
      const cx<R>* cb = B + (2 * f + 1) * M;
      za = spec_value<R>(kind, n, m, half, [&](int k) { return ca[k]; });
      zb = spec_value<R>(kind, n, m, half, [&](int k) { return cb[k]; });
    } else {
      const R* ra = (const R*)B + (2 * f) * M;
      const R* rb = (const R*)B + (2 * f + 1) * M;
      za = spec_value<R>(kind, n, m, false, [&](int k) { return mk<R>(ra[k], (R)0); });
      zb = spec_value<R>(kind, n, m, false, [&](int k) { return mk<R>(rb[k], (R)0); });
    }
    A[f * LS + m] = mk<R>(za.re - zb.im, za.im + zb.re);   // za + i zb
  }
  __syncthreads();
  const cx<R>* Z = lds_fft<R>(A, B, F, L, LS, d.nrad, d.rad, (const cx<R>*)d.tw, true);
  const R invL = (R)1 / (R)L;
  const int Nx = d.len_out;   // n + 1 nodes
  const int nb = C->n_b;
  R be[MAX_DEPTH];
  const R* dsrc[MAX_DEPTH];
  for (int t = 0; t < MAX_DEPTH; ++t) {
    be[t] = t < nb ? (R)C->beta[t] : (R)0;
    dsrc[t] = (const R*)d.ring + (int64_t)(t < nb ? C->slot_b[t] : 0) * d.ring_stride;
  }
  R* dw = (R*)d.ring + (int64_t)C->slot_w * d.ring_stride;
  for (int idx = threadIdx.x; idx < nrows * Nx; idx += blockDim.x) {
    const int r = idx / Nx, j = idx - r * Nx;
    const int x = node_src(kind, n, j);
    R v = 0;
    if (x >= 0) {
      const cx<R> z = Z[(r >> 1) * LS + x];
      v = ((r & 1) ? z.im : z.re) * invL;
    }
    const int64_t o = (int64_t)(row0 + r) * d.out_s1 + j;
    R dl = v;
    for (int t = 0; t < nb; ++t) dl -= be[t] * dsrc[t][o];
    dw[o] = dl;
    d.uf[o] += (double)dl;
  }
}

// ---------------------------------------------------------------------------
template <typename R, int MODE>
__global__ void __launch_bounds__(256) k_strided(const PassDesc* __restrict__ descs, const int2* __restrict__ work,
                                                 const SolveDev* __restrict__ S) {
  extern __shared__ __align__(16) char smem[];
  const int2 w = work[blockIdx.x];
  const PassDesc& d = descs[w.x];
  const Ctrl* C = S[d.solve].ctrl;
  if (C->status != ST_RUNNING) return;
  const int L = d.L, LS = L + 4, F = d.F, n = d.n, kind = d.kind;
  cx<R>* A = (cx<R>*)smem;
  cx<R>* B = A + F * LS;
  const int cols = d.cols;
  const int tp = w.y % d.tiles_p0;
  const int p1 = w.y / d.tiles_p0;
  const int p0b = tp * cols;
  const int ncol = min(cols, d.n_p0 - p0b);
  const bool packed = d.packed;
  const cx<R>* W = (const cx<R>*)d.tw;
  const cx<R>* Z;
  int M;     // coefficient count along the axis
  bool half; // r2c-halved DFT (real data along a periodic axis)
  half = packed && kind == K_DFT;
  M = half ? n / 2 + 1 : n_freq(kind, n);

  if (MODE == 0 || MODE == 2) {
    int j0, cnt;
    raw_range(kind, n, j0, cnt);
    if (!d.cplx_in) {
      R* raw = (R*)B;
      for (int idx = threadIdx.x; idx < cols * cnt; idx += blockDim.x) {
        const int c = idx % cols, e = idx / cols;
        R v = 0;
        if (c < ncol) v = ((const R*)d.in)[(int64_t)(p0b + c) + (int64_t)(j0 + e) * d.in_sa + (int64_t)p1 * d.in_s1];
        raw[c * cnt + e] = v;
      }
    } else {
      for (int idx = threadIdx.x; idx < cols * cnt; idx += blockDim.x) {
        const int c = idx % cols, e = idx / cols;
        cx<R> v = mk<R>(0, 0);
        if (c < ncol) v = ldc<R>(d.in, (int64_t)(p0b + c) + (int64_t)(j0 + e) * d.in_sa + (int64_t)p1 * d.in_s1);
        B[c * cnt + e] = v;
      }
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < F * L; idx += blockDim.x) {
      const int f = idx / L, x = idx - f * L;
      int j, sg;
      ext_src(kind, n, x, j, sg);
      cx<R> v = mk<R>(0, 0);
      if (sg) {
        if (packed) {
          const R* raw = (const R*)B;
          v = mk<R>((R)sg * raw[(2 * f) * cnt + (j - j0)], (R)sg * raw[(2 * f + 1) * cnt + (j - j0)]);
        } else {
          v = scl(B[f * cnt + (j - j0)], (R)sg);
        }
      }
      A[f * LS + x] = v;
    }
    __syncthreads();
    Z = lds_fft<R>(A, B, F, L, LS, d.nrad, d.rad, W, false);
    if (MODE == 0) {
      for (int idx = threadIdx.x; idx < cols * M; idx += blockDim.x) {
        const int c = idx % cols, k = idx / cols;
        if (c >= ncol) continue;
        const cx<R> v = packed ? fwd_coef<R>(Z + (c >> 1) * LS, L, kind, k, 1, c & 1)
                               : fwd_coef<R>(Z + c * LS, L, kind, k, 0, 0);
        const int64_t o = (int64_t)(p0b + c) + (int64_t)k * d.out_sa + (int64_t)p1 * d.out_s1;
        if (d.cplx_out) stc<R>(d.out, o, v);
        else ((R*)d.out)[o] = v.re;
      }
      return;
    }
    // MODE 2: coefficients times the Green factor into the other buffer
    cx<R>* coef = (Z == A) ? B : A;
    cx<R>* zbuf = (Z == A) ? A : B;
    const bool realc = packed && !half;
    for (int idx = threadIdx.x; idx < cols * M; idx += blockDim.x) {
      const int c = idx % cols, k = idx / cols;
      cx<R> v = packed ? fwd_coef<R>(Z + (c >> 1) * LS, L, kind, k, 1, c & 1)
                       : fwd_coef<R>(Z + c * LS, L, kind, k, 0, 0);
      const double g = (c < ncol) ? green_factor(d, p0b + c, p1, k) : 0.0;
      v = scl(v, (R)g);
      if (realc) ((R*)coef)[c * M + k] = v.re;
      else coef[c * M + k] = v;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < F * L; idx += blockDim.x) {
      const int f = idx / L, m = idx - f * L;
      cx<R> v;
      if (realc) {
        const R* ra = (const R*)coef + (2 * f) * M;
        const R* rb = (const R*)coef + (2 * f + 1) * M;
        const cx<R> za = spec_value<R>(kind, n, m, false, [&](int k) { return mk<R>(ra[k], (R)0); });
        const cx<R> zb = spec_value<R>(kind, n, m, false, [&](int k) { return mk<R>(rb[k], (R)0); });
        v = mk<R>(za.re - zb.im, za.im + zb.re);
      } else if (packed) {   // half: two Hermitian spectra
        const cx<R>* ca = coef + (2 * f) * M;
        const cx<R>* cb = coef + (2 * f + 1) * M;
        const cx<R> za = spec_value<R>(kind, n, m, true, [&](int k) { return ca[k]; });
        const cx<R> zb = spec_value<R>(kind, n, m, true, [&](int k) { return cb[k]; });
        v = mk<R>(za.re - zb.im, za.im + zb.re);
      } else {
        const cx<R>* cc = coef + f * M;
        v = spec_value<R>(kind, n, m, false, [&](int k) { return cc[k]; });
      }
      zbuf[f * LS + m] = v;
    }
    __syncthreads();
    Z = lds_fft<R>(zbuf, coef, F, L, LS, d.nrad, d.rad, W, true);
  } else {
    // MODE 1: inverse from coefficients
    const int Min = d.len_in;
    if (!d.cplx_in) {
      R* raw = (R*)B;
      for (int idx = threadIdx.x; idx < cols * Min; idx += blockDim.x) {
        const int c = idx % cols, k = idx / cols;
        R v = 0;
        if (c < ncol) v = ((const R*)d.in)[(int64_t)(p0b + c) + (int64_t)k * d.in_sa + (int64_t)p1 * d.in_s1];
        raw[c * Min + k] = v;
      }
    } else {
      for (int idx = threadIdx.x; idx < cols * Min; idx += blockDim.x) {
        const int c = idx % cols, k = idx / cols;
        cx<R> v = mk<R>(0, 0);
        if (c < ncol) v = ldc<R>(d.in, (int64_t)(p0b + c) + (int64_t)k * d.in_sa + (int64_t)p1 * d.in_s1);
        B[c * Min + k] = v;
      }
    }
    __syncthreads();
    // inverse packing: real output <=> packed
    const bool ihalf = packed && kind == K_DFT;
    for (int idx = threadIdx.x; idx < F * L; idx += blockDim.x) {
      const int f = idx / L, m = idx - f * L;
      cx<R> v;
      if (packed && !d.cplx_in) {
        const R* ra = (const R*)B + (2 * f) * Min;
        const R* rb = (const R*)B + (2 * f + 1) * Min;
        const cx<R> za = spec_value<R>(kind, n, m, false, [&](int k) { return mk<R>(ra[k], (R)0); });
        const cx<R> zb = spec_value<R>(kind, n, m, false, [&](int k) { return mk<R>(rb[k], (R)0); });
        v = mk<R>(za.re - zb.im, za.im + zb.re);
      } else if (packed) {
        const cx<R>* ca = B + (2 * f) * Min;
        const cx<R>* cb = B + (2 * f + 1) * Min;
        const cx<R> za = spec_value<R>(kind, n, m, ihalf, [&](int k) { return ca[k]; });
        const cx<R> zb = spec_value<R>(kind, n, m, ihalf, [&](int k) { return cb[k]; });
        v = mk<R>(za.re - zb.im, za.im + zb.re);
      } else {
        const cx<R>* cc = B + f * Min;
        v = spec_value<R>(kind, n, m, false, [&](int k) { return cc[k]; });
      }
      A[f * LS + m] = v;
    }
    __syncthreads();
    Z = lds_fft<R>(A, B, F, L, LS, d.nrad, d.rad, W, true);
  }
  // store node values along the axis (MODE 1 and 2)
  const R invL = (R)1 / (R)L;
  const int Nout = n + 1;
  for (int idx = threadIdx.x; idx < cols * Nout; idx += blockDim.x) {
    const int c = idx % cols, j = idx / cols;
    if (c >= ncol) continue;
    const int x = node_src(kind, n, j);
    const int64_t o = (int64_t)(p0b + c) + (int64_t)j * d.out_sa + (int64_t)p1 * d.out_s1;
    if (packed) {
      R v = 0;
      if (x >= 0) {
        const cx<R> z = Z[(c >> 1) * LS + x];
        v = ((c & 1) ? z.im : z.re) * invL;
      }
      ((R*)d.out)[o] = v;
    } else {
      cx<R> v = mk<R>(0, 0);
      if (x >= 0) v = scl(Z[c * LS + x], invL);
      stc<R>(d.out, o, v);
    }
  }
}

}  // namespace fm

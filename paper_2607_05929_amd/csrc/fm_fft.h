// LDS pencil transforms: every Table 1 transform (DFT, DCT-I, DST-I, DCT-III,
// DST-III) of a pencil is evaluated as a complex FFT of length L of the
// virtually extended field (L = n, 2n or 4n = S_f n, Sec. 2.4), computed by a
// mixed-radix Stockham pass sequence in LDS.  Two real pencils share one
// complex FFT (real and imaginary parts) and are separated afterwards with
// the conjugate-symmetry identities; complex pencils (after a DFT axis) use
// one FFT each.  The extension is built in LDS and never written to HBM.
#pragma once
#include "fm_common.h"

namespace fm {

template <typename R> struct cx { R re, im; };

template <typename R> __device__ __forceinline__ cx<R> mk(R a, R b) { cx<R> z; z.re = a; z.im = b; return z; }
template <typename R> __device__ __forceinline__ cx<R> add(cx<R> a, cx<R> b) { return mk<R>(a.re + b.re, a.im + b.im); }
template <typename R> __device__ __forceinline__ cx<R> sub(cx<R> a, cx<R> b) { return mk<R>(a.re - b.re, a.im - b.im); }
template <typename R> __device__ __forceinline__ cx<R> mul(cx<R> a, cx<R> b) {
  return mk<R>(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename R> __device__ __forceinline__ cx<R> scl(cx<R> a, R s) { return mk<R>(a.re * s, a.im * s); }
template <typename R> __device__ __forceinline__ cx<R> conj(cx<R> a) { return mk<R>(a.re, -a.im); }
// multiply by (sgn * i)
template <typename R> __device__ __forceinline__ cx<R> mul_si(cx<R> a, R sgn) { return mk<R>(-sgn * a.im, sgn * a.re); }

// Twiddle lookup: exp(sgn 2 pi i t / L) from the forward table W[t] = exp(-2 pi i t / L).
template <typename R> __device__ __forceinline__ cx<R> twid(const cx<R>* W, int t, bool inv) {
  cx<R> w = W[t];
  return inv ? conj(w) : w;   // forward uses the table value exp(-2 pi i t / L)
}
// Global loads and stores at a 32-bit byte offset from a wavefront-uniform
// base: the address is the scalar base plus one zero-extended VGPR, with no
// 64-bit arithmetic per access.  Complex values move as one 2-wide access.
template <typename T>
__device__ __forceinline__ T gld(const FM_GLOBAL char* base, uint32_t off) {
  return *(const FM_GLOBAL T*)(base + off);
}
template <typename T>
__device__ __forceinline__ void gst(FM_GLOBAL char* base, uint32_t off, T v) {
  *(FM_GLOBAL T*)(base + off) = v;
}
template <typename R>
__device__ __forceinline__ cx<R> gldc(const FM_GLOBAL char* base, uint32_t off) {
  typedef R R2 __attribute__((ext_vector_type(2)));
  const R2 v = gld<R2>(base, off);
  return mk<R>(v.x, v.y);
}
template <typename R>
__device__ __forceinline__ void gstc(FM_GLOBAL char* base, uint32_t off, cx<R> c) {
  typedef R R2 __attribute__((ext_vector_type(2)));
  R2 v;
  v.x = c.re; v.y = c.im;
  gst<R2>(base, off, v);
}

// LDS views (address space 3): ds instructions, counted by the LDS counter
// only, so that waits on them do not wait for global loads in flight.
#define FM_LDS __attribute__((address_space(3)))
template <typename R> __device__ __forceinline__ cx<R> twid(const FM_LDS cx<R>* W, int t, bool inv) {
  typedef R R2 __attribute__((ext_vector_type(2)));
  const R2 v = *(const FM_LDS R2*)(W + t);
  return inv ? mk<R>(v.x, -v.y) : mk<R>(v.x, v.y);
}

template <typename R> __device__ __forceinline__ cx<R> twid(const FM_GLOBAL cx<R>* W, int t, bool inv) {
  const cx<R> w = gldc<R>((const FM_GLOBAL char*)W, (uint32_t)t * (uint32_t)sizeof(cx<R>));
  return inv ? conj(w) : w;
}

template <typename R> __device__ __forceinline__ void bfly2(cx<R>* u) {
  cx<R> a = u[0], b = u[1];
  u[0] = add(a, b); u[1] = sub(a, b);
}

template <typename R> __device__ __forceinline__ void bfly4(cx<R>* u, R sgn) {
  cx<R> a = add(u[0], u[2]), b = sub(u[0], u[2]);
  cx<R> c = add(u[1], u[3]), d = mul_si(sub(u[1], u[3]), sgn);
  u[0] = add(a, c); u[2] = sub(a, c); u[1] = add(b, d); u[3] = sub(b, d);
}

template <typename R> __device__ __forceinline__ void bfly8(cx<R>* u, R sgn) {
  cx<R> e[4] = {u[0], u[2], u[4], u[6]};
  cx<R> o[4] = {u[1], u[3], u[5], u[7]};
  bfly4(e, sgn); bfly4(o, sgn);
  const R r2 = (R)0.70710678118654752440;
  // w8^s = exp(sgn 2 pi i s / 8)
  cx<R> w1 = mk<R>(r2, sgn * r2), w3 = mk<R>(-r2, sgn * r2);
  cx<R> t0 = o[0], t1 = mul(o[1], w1), t2 = mul_si(o[2], sgn), t3 = mul(o[3], w3);
  u[0] = add(e[0], t0); u[4] = sub(e[0], t0);
  u[1] = add(e[1], t1); u[5] = sub(e[1], t1);
  u[2] = add(e[2], t2); u[6] = sub(e[2], t2);
  u[3] = add(e[3], t3); u[7] = sub(e[3], t3);
}

template <typename R> __device__ __forceinline__ void bfly3(cx<R>* u, R sgn) {
  const R h3 = (R)0.86602540378443864676;
  cx<R> s = add(u[1], u[2]);
  cx<R> t1 = sub(u[0], scl(s, (R)0.5));
  cx<R> t2 = mul_si(scl(sub(u[1], u[2]), h3), sgn);
  u[0] = add(u[0], s); u[1] = add(t1, t2); u[2] = sub(t1, t2);
}

template <typename R> __device__ __forceinline__ void bfly5(cx<R>* u, R sgn) {
  const R c1 = (R)0.30901699437494742410, c2 = (R)-0.80901699437494742410;
  const R s1 = (R)0.95105651629515357212, s2 = (R)0.58778525229247312917;
  cx<R> a1 = add(u[1], u[4]), b1 = sub(u[1], u[4]);
  cx<R> a2 = add(u[2], u[3]), b2 = sub(u[2], u[3]);
  cx<R> r1 = add(u[0], add(scl(a1, c1), scl(a2, c2)));
  cx<R> r2 = add(u[0], add(scl(a1, c2), scl(a2, c1)));
  cx<R> i1 = mul_si(add(scl(b1, s1), scl(b2, s2)), sgn);
  cx<R> i2 = mul_si(sub(scl(b1, s2), scl(b2, s1)), sgn);
  u[0] = add(u[0], add(a1, a2));
  u[1] = add(r1, i1); u[4] = sub(r1, i1);
  u[2] = add(r2, i2); u[3] = sub(r2, i2);
}

// One Stockham autosort stage over F pencils of length L stored with stride L:
// butterfly i (0 <= i < L/R) reads x[i + r L/R], twiddles by
// exp(sgn 2 pi i r k / (p R)) with k = i mod p, transforms with radix R and
// writes y[(i - k) R + k + s p].  After all stages (p = product of radices
// so far) the output is the DFT in natural order.
template <typename R, int RAD>
__device__ __forceinline__ void stage_fixed(const cx<R>* __restrict__ src, cx<R>* __restrict__ dst,
                                            int F, int L, int LS, int p, const cx<R>* W, bool inv) {
  const int T = L / RAD;
  const int tstep = L / (p * RAD);
  const R sgn = inv ? (R)1 : (R)-1;
  for (int b = threadIdx.x; b < F * T; b += blockDim.x) {
    const int f = b / T, i = b - f * T;
    const int k = i % p;
    const cx<R>* s = src + f * LS;
    cx<R> u[RAD];
#pragma unroll
    for (int r = 0; r < RAD; ++r) {
      cx<R> v = s[i + r * T];
      if (r > 0 && k > 0) v = mul(v, twid(W, r * k * tstep, inv));
      u[r] = v;
    }
    if constexpr (RAD == 2) bfly2(u);
    else if constexpr (RAD == 3) bfly3(u, sgn);
    else if constexpr (RAD == 4) bfly4(u, sgn);
    else if constexpr (RAD == 5) bfly5(u, sgn);
    else bfly8(u, sgn);
    cx<R>* d = dst + f * LS + (i - k) * RAD + k;
#pragma unroll
    for (int s2 = 0; s2 < RAD; ++s2) d[s2 * p] = u[s2];
  }
}

// Any other radix: direct O(R^2) butterfly read from LDS.
template <typename R>
__device__ __forceinline__ void stage_generic(const cx<R>* __restrict__ src, cx<R>* __restrict__ dst,
                                              int F, int L, int LS, int p, int RAD, const cx<R>* W, bool inv) {
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
      cx<R> v = s[i + r * T];
      if (r > 0 && k > 0) v = mul(v, twid(W, r * k * tstep, inv));
      const int e = (r * s2) % RAD;
      if (e) v = mul(v, twid(W, e * T, inv));
      acc = add(acc, v);
    }
    dst[f * LS + (i - k) * RAD + k + s2 * p] = acc;
  }
}

// Full FFT of F pencils; data starts in a, b is scratch; returns the buffer
// holding the result.  Caller synchronises before; this synchronises after.
template <typename R>
__device__ cx<R>* lds_fft(cx<R>* a, cx<R>* b, int F, int L, int LS, int nrad, const int32_t* rad,
                          const cx<R>* W, bool inv) {
  int p = 1;
  for (int st = 0; st < nrad; ++st) {
    const int RAD = rad[st];
    switch (RAD) {
      case 2: stage_fixed<R, 2>(a, b, F, L, LS, p, W, inv); break;
      case 3: stage_fixed<R, 3>(a, b, F, L, LS, p, W, inv); break;
      case 4: stage_fixed<R, 4>(a, b, F, L, LS, p, W, inv); break;
      case 5: stage_fixed<R, 5>(a, b, F, L, LS, p, W, inv); break;
      case 8: stage_fixed<R, 8>(a, b, F, L, LS, p, W, inv); break;
      default: stage_generic<R>(a, b, F, L, LS, p, RAD, W, inv); break;
    }
    __syncthreads();
    cx<R>* t = a; a = b; b = t;
    p *= RAD;
  }
  return a;
}

// ---------------------------------------------------------------------------
// Extensions (Table 1, Fig. Symmetries)
// ---------------------------------------------------------------------------
// Forward raw-load range of node indices along an axis: [j0, j0 + cnt).
__host__ __device__ inline void raw_range(int kind, int n, int& j0, int& cnt) {
  switch (kind) {
    case K_DFT:  j0 = 0; cnt = n; break;
    case K_DCT1: j0 = 0; cnt = n + 1; break;
    case K_DST1: j0 = 1; cnt = n - 1; break;
    case K_DCT3: j0 = 0; cnt = n; break;
    default:     j0 = 1; cnt = n; break;   // DST3
  }
}

__host__ __device__ inline int n_freq(int kind, int n) {
  switch (kind) {
    case K_DFT: return n;
    case K_DCT1: return n + 1;
    case K_DST1: return n - 1;
    default: return n;
  }
}

// Extension factor S_f of a kind (L = S_f n).
__host__ __device__ constexpr int kind_sf(int kind) {
  return kind == K_DFT ? 1 : ((kind == K_DCT1 || kind == K_DST1) ? 2 : 4);
}

__host__ __device__ inline int ext_len(int kind, int n) {
  return kind == K_DFT ? n : ((kind == K_DCT1 || kind == K_DST1) ? 2 * n : 4 * n);
}

// Position x of the extended field E -> node index j and sign (0 = zero).
__device__ __forceinline__ void ext_src(int kind, int n, int x, int& j, int& sg) {
  sg = 1; j = 0;
  switch (kind) {
    case K_DFT: j = x; return;
    case K_DCT1: j = x <= n ? x : 2 * n - x; return;
    case K_DST1:
      if (x == 0 || x == n) { sg = 0; return; }
      if (x < n) { j = x; } else { j = 2 * n - x; sg = -1; }
      return;
    case K_DCT3: {
      const int y = x <= 2 * n ? x : 4 * n - x;
      if (y < n) { j = y; } else if (y == n) { sg = 0; } else { j = 2 * n - y; sg = -1; }
      return;
    }
    default: {  // DST3
      int y = x;
      if (x > 2 * n) { y = 4 * n - x; sg = -1; }
      if (y == 0 || y == 2 * n) { sg = 0; return; }
      j = y <= n ? y : 2 * n - y;
      return;
    }
  }
}

// Extended spectrum position m -> coefficient index k and factor
// (DFT(E)[map(k)] = alpha DT(G)[k], Table 1, extended by the spectrum's own
// parity).  Factor encoded as (fr, fi) complex.
template <typename R>
__device__ __forceinline__ bool spec_src(int kind, int n, int m, int& k, R& fr, R& fi) {
  fr = 1; fi = 0; k = m;
  switch (kind) {
    case K_DFT: return true;
    case K_DCT1: k = m <= n ? m : 2 * n - m; return true;
    case K_DST1:
      if (m == 0 || m == n) return false;
      if (m < n) { k = m - 1; fr = 0; fi = -1; } else { k = 2 * n - m - 1; fr = 0; fi = 1; }
      return true;
    case K_DCT3:
      if ((m & 1) == 0) return false;
      k = m < 2 * n ? (m - 1) / 2 : (4 * n - m - 1) / 2; fr = 2; fi = 0;
      return true;
    default:
      if ((m & 1) == 0) return false;
      if (m < 2 * n) { k = (m - 1) / 2; fr = 0; fi = -2; } else { k = (4 * n - m - 1) / 2; fr = 0; fi = 2; }
      return true;
  }
}

// Forward extraction: coefficient k <- extended spectrum index and 1/alpha.
template <typename R>
__device__ __forceinline__ void coef_src(int kind, int k, int& m, R& fr, R& fi) {
  switch (kind) {
    case K_DFT:
    case K_DCT1: m = k; fr = 1; fi = 0; return;
    case K_DST1: m = k + 1; fr = 0; fi = 1; return;          // 1/(-i) = i
    case K_DCT3: m = 2 * k + 1; fr = (R)0.5; fi = 0; return;
    default: m = 2 * k + 1; fr = 0; fi = (R)0.5; return;     // 1/(-2i) = i/2
  }
}

// Inverse output: node j <- extended real-space position (or zero).
__device__ __forceinline__ int node_src(int kind, int n, int j) {
  switch (kind) {
    case K_DFT: return j == n ? 0 : j;
    case K_DCT1: return j;
    case K_DST1: return (j == 0 || j == n) ? -1 : j;
    case K_DCT3: return j == n ? -1 : j;
    default: return j == 0 ? -1 : j;
  }
}

}  // namespace fm

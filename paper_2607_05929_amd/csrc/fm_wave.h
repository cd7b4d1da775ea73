// Wavefront-per-pencil axis passes for pencil lengths L = 64 E (E in
// {1, 2, 3, 4, 5, 6, 8, 12, 16}), the common case of the solver's grids,
// and half- / quarter-wavefront forms for L = 32 E and 16 E (E in {1, 3}):
// LN = 32 or 16 lanes per pencil, two or four pencils per wavefront, so
// that the 32-, 48- and 96-point pencils of small grids also take the
// register transform instead of the generic LDS kernel.
//
// A block of 8 wavefronts owns a tile of 8 * 64 / LN pencils (two real
// columns packed per pencil, or one complex column: 16 or 8 columns at
// LN = 64): small blocks so that several fit a compute unit and one block's
// loads overlap another's arithmetic.  The tile is loaded with coalesced row
// segments (64 bytes at LN = 64; whole rows along x) into an LDS staging
// array; each group of LN lanes then gathers its pencil's virtual
// extension (Table 1) straight into registers, lane t holding positions
// t + LN j (j < E), and transforms it with
//   X[k1 + E k2] = sum_t W_L^{t k1} W_LN^{t k2} sum_j x[t + LN j] W_E^{j k1}:
// an E-point DFT in registers, a twiddle, and an LN-point DFT across the
// lanes (radix-2 butterflies through lane exchanges, decimation in frequency
// forward and in time inverse, so the spectrum stays in bit-reversed lane
// order and needs no reordering).  The Green operator of the fused z pass
// scales the spectrum in registers.  Results go back through the staging
// array to coalesced stores.  No block barrier separates FFT stages; the
// staging array is the only LDS.
#pragma once
#include <type_traits>
#include "fm_pass.h"

namespace fm {

constexpr int WAVE_PENCILS = 8;         // wavefronts per block (its pencils at 64 lanes per pencil)
constexpr int WAVE_THREADS = 64 * WAVE_PENCILS;

__host__ __device__ inline bool wave_E_ok(int E) {
  return E == 1 || E == 2 || E == 3 || E == 4 || E == 5 || E == 6 || E == 8 || E == 12 || E == 16;
}

template <typename R>
__device__ __forceinline__ cx<R> shfl_xor_c(cx<R> v, int m) {
  return mk<R>(__shfl_xor(v.re, m, 64), __shfl_xor(v.im, m, 64));
}
template <typename R>
__device__ __forceinline__ cx<R> shfl_c(cx<R> v, int src) {
  return mk<R>(__shfl(v.re, src, 64), __shfl(v.im, src, 64));
}

__device__ __forceinline__ int brev6(int x) { return (int)(__brev((unsigned)x) >> 26); }

constexpr int lanes_log2(int LN) { return LN == 64 ? 6 : LN == 32 ? 5 : 4; }

// Bit reversal of an LN-lane index.
template <int LN>
__device__ __forceinline__ int brev_ln(int x) { return (int)(__brev((unsigned)x) >> (32 - lanes_log2(LN))); }

// Per-lane constants of the LN-point lane DFT (stages ST = log2 LN).  Stage i
// pairs lanes that differ in bit h = LN / 2 >> i; sg[i] is +1 on the lane
// with the bit clear and -1 on the lane with it set, s[i] is W_{2h}^{lane mod
// h} on the lane with the bit set and 1 on the other (forward values; the
// inverse uses conjugates).  They depend on the lane only and are loaded once
// per pencil pass.
template <typename R, int LN = 64>
struct LaneTw {
  static constexpr int ST = lanes_log2(LN);
  cx<R> s[ST - 1];
  R sg[ST];
};

template <typename R, int LN>
__device__ __forceinline__ LaneTw<R, LN> lane_twiddles(const FM_GLOBAL cx<R>* W, int L) {
  constexpr int ST = lanes_log2(LN);
  const int lane = threadIdx.x & (LN - 1);
  LaneTw<R, LN> tw;
#pragma unroll
  for (int i = 0; i < ST; ++i) {
    const int h = (LN / 2) >> i;
    tw.sg[i] = (lane & h) ? (R)-1 : (R)1;
    if (i < ST - 1) tw.s[i] = (lane & h) ? twid<R>(W, (lane & (h - 1)) * (L / (2 * h)), false) : mk<R>(1, 0);
  }
  return tw;
}

// Forward LN-point DFT across the lanes of every register (each group of LN
// lanes on its own), decimation in frequency: lane t starts with x[t] and
// ends with X[brev(t)].  Stages are the outer loop so that the exchanges of
// all registers are in flight together; the butterflies are branch free
// (sign and twiddle per lane).
template <typename R, int E, int LN>
__device__ __forceinline__ void lane_dif(cx<R> (&v)[E], const LaneTw<R, LN>& tw) {
  constexpr int ST = lanes_log2(LN);
#pragma unroll
  for (int i = 0; i < ST; ++i) {
    const int h = (LN / 2) >> i;
    cx<R> pv[E];
#pragma unroll
    for (int k = 0; k < E; ++k) pv[k] = shfl_xor_c(v[k], h);
#pragma unroll
    for (int k = 0; k < E; ++k) {
      cx<R> z = mk<R>(fma(tw.sg[i], v[k].re, pv[k].re), fma(tw.sg[i], v[k].im, pv[k].im));
      if (i < ST - 1) z = mul(z, tw.s[i]);
      v[k] = z;
    }
  }
}

// Inverse LN-point DFT across the lanes (unnormalised), decimation in time:
// lane t starts with X[brev(t)] and ends with x[t].
template <typename R, int E, int LN>
__device__ __forceinline__ void lane_dit(cx<R> (&v)[E], const LaneTw<R, LN>& tw) {
  constexpr int ST = lanes_log2(LN);
#pragma unroll
  for (int i = ST - 1; i >= 0; --i) {
    const int h = (LN / 2) >> i;
    if (i < ST - 1) {
#pragma unroll
      for (int k = 0; k < E; ++k) v[k] = mul(v[k], conj(tw.s[i]));
    }
    cx<R> pv[E];
#pragma unroll
    for (int k = 0; k < E; ++k) pv[k] = shfl_xor_c(v[k], h);
#pragma unroll
    for (int k = 0; k < E; ++k)
      v[k] = mk<R>(fma(tw.sg[i], v[k].re, pv[k].re), fma(tw.sg[i], v[k].im, pv[k].im));
  }
}

// In-register E-point DFT (natural order in and out).
template <typename R, int E>
__device__ __forceinline__ void dft_reg(cx<R> (&v)[E], const FM_GLOBAL cx<R>* W, int L, bool inv) {
  const R sgn = inv ? (R)1 : (R)-1;
  if constexpr (E == 1) {
    return;
  } else if constexpr (E == 2) {
    bfly2(v);
  } else if constexpr (E == 3) {
    bfly3(v, sgn);
  } else if constexpr (E == 4) {
    bfly4(v, sgn);
  } else if constexpr (E == 5) {
    bfly5(v, sgn);
  } else if constexpr (E == 8) {
    bfly8(v, sgn);
  } else {
    // E = A B: A-point DFTs over j = B ja + jb, twiddle W_E^{jb ka}, B-point DFTs
    constexpr int A = (E == 6) ? 2 : (E == 12) ? 4 : 4;   // 6 = 2x3, 12 = 4x3, 16 = 4x4
    constexpr int B = E / A;
    cx<R> y[B][A];
#pragma unroll
    for (int jb = 0; jb < B; ++jb) {
#pragma unroll
      for (int ja = 0; ja < A; ++ja) y[jb][ja] = v[B * ja + jb];
      if constexpr (A == 2) bfly2(y[jb]);
      else bfly4(y[jb], sgn);
#pragma unroll
      for (int ka = 1; ka < A; ++ka)
        if (jb) y[jb][ka] = mul(y[jb][ka], twid(W, (jb * ka) * (L / E), inv));
    }
#pragma unroll
    for (int ka = 0; ka < A; ++ka) {
      cx<R> z[B];
#pragma unroll
      for (int jb = 0; jb < B; ++jb) z[jb] = y[jb][ka];
      if constexpr (B == 3) bfly3(z, sgn);
      else bfly4(z, sgn);
#pragma unroll
      for (int kb = 0; kb < B; ++kb) v[ka + A * kb] = z[kb];
    }
  }
}

// Forward: lane t (of LN) holds x[t + LN j] in v[j]; on return lane t holds
// X[k1 + E brev(t)] in v[k1].  Inverse: the exact mirror image (input in
// that bit-reversed layout, output x[t + LN j] in v[j], unnormalised).
template <typename R, int E, int LN>
__device__ __forceinline__ void wave_fft(cx<R> (&v)[E], const FM_GLOBAL cx<R>* W, const LaneTw<R, LN>& tw,
                                         bool inv) {
  constexpr int L = LN * E;
  const int t = threadIdx.x & (LN - 1);
  if (!inv) {
    dft_reg<R, E>(v, W, L, false);
#pragma unroll
    for (int k1 = 1; k1 < E; ++k1) v[k1] = mul(v[k1], twid<R>(W, t * k1, false));
    lane_dif<R, E, LN>(v, tw);
  } else {
    lane_dit<R, E, LN>(v, tw);
#pragma unroll
    for (int k1 = 1; k1 < E; ++k1) v[k1] = mul(v[k1], twid<R>(W, t * k1, true));
    dft_reg<R, E>(v, W, L, true);
  }
}

// E = 8 (L = 512), the grids' common case: the 64-point DFT over the lanes
// is split 8 x 8 through two in-wave transposes in LDS, so that every
// butterfly is a radix-8 in registers (no lane exchanges, no idle half).
// Lane t = a + 8 b = c + 8 k1; with n = a + 8 b + 64 j and
// m = k1 + 8 c + 64 d,
//   X[m] = sum_a W_8^{a d} W_64^{a c} sum_b W_8^{b c} W_512^{(a + 8 b) k1}
//          sum_j W_8^{j k1} x[n].
// Forward: lane t holds x[t + 64 j] in v[j]; on return lane t holds
// X[(t >> 3) + 8 (t & 7) + 64 d] in v[d].  Inverse: the exact mirror image
// (unnormalised).  The scratch of one wave is WT_SIZE reals; the two index
// maps are conflict-free on the 64 LDS banks for both access orders.
constexpr int WT_PITCH = 72, WT_SIZE = 8 * WT_PITCH;

template <typename R, typename WI, typename RI>
__device__ __forceinline__ void wave_xpose(R* sb, cx<R> (&v)[8], WI widx, RI ridx) {
  R tmp[8];
#pragma unroll
  for (int part = 0; part < 2; ++part) {
#pragma unroll
    for (int r = 0; r < 8; ++r) sb[widx(r)] = part ? v[r].im : v[r].re;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int r = 0; r < 8; ++r) tmp[r] = sb[ridx(r)];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      if (part) v[r].im = tmp[r];
      else v[r].re = tmp[r];
    }
  }
}

// Twiddles of the E = 8 transform: the first stage takes W_512^(t k1)
// (k1 = 1..7), the second W_64^(lo c) = W_512^(8 lo c) (c = 1..7).  From the
// global L-table, or from an LDS table laid out per stage so that the reads
// of a wavefront are conflict-free: [k1 - 1][t] (448 entries), then
// [c - 1][lo] (56 entries, read as broadcasts).
constexpr int TW8_LDS = 7 * 64 + 7 * 8;
template <typename R>
struct TwGlobal {
  const FM_GLOBAL cx<R>* W;
  __device__ __forceinline__ cx<R> s1(int t, int k1, bool inv) const { return twid<R>(W, t * k1, inv); }
  __device__ __forceinline__ cx<R> s2(int lo, int c, bool inv) const { return twid<R>(W, 8 * lo * c, inv); }
};
template <typename R>
struct TwLds {
  const FM_LDS cx<R>* T;
  __device__ __forceinline__ cx<R> s1(int t, int k1, bool inv) const { return twid<R>(T, (k1 - 1) * 64 + t, inv); }
  __device__ __forceinline__ cx<R> s2(int lo, int c, bool inv) const {
    return twid<R>(T, 7 * 64 + (c - 1) * 8 + lo, inv);
  }
};

template <typename R, typename TW>
__device__ __forceinline__ void wave_fft8(cx<R> (&v)[8], const TW& W, R* sb, bool inv) {
  const int t = threadIdx.x & 63;
  const int lo = t & 7, hi = t >> 3;
  auto t1_w = [&](int r) { return WT_PITCH * r + t; };                  // lane a + 8 b, register k1
  auto t1_r = [&](int r) { return WT_PITCH * hi + lo + 8 * r; };        // lane a + 8 k1, register b
  auto t2_w = [&](int r) { return WT_PITCH * hi + 9 * r + lo; };        // lane a + 8 k1, register c
  auto t2_r = [&](int r) { return WT_PITCH * hi + 9 * lo + r; };        // lane c + 8 k1, register a
  const R sgn = inv ? (R)1 : (R)-1;
  if (!inv) {
    bfly8(v, sgn);                                                      // j -> k1
#pragma unroll
    for (int k1 = 1; k1 < 8; ++k1) v[k1] = mul(v[k1], W.s1(t, k1, false));
    wave_xpose<R>(sb, v, t1_w, t1_r);
    bfly8(v, sgn);                                                      // b -> c
#pragma unroll
    for (int c = 1; c < 8; ++c) v[c] = mul(v[c], W.s2(lo, c, false));
    wave_xpose<R>(sb, v, t2_w, t2_r);
    bfly8(v, sgn);                                                      // a -> d
  } else {
    bfly8(v, sgn);                                                      // d -> a
    wave_xpose<R>(sb, v, t2_r, t2_w);
#pragma unroll
    for (int c = 1; c < 8; ++c) v[c] = mul(v[c], W.s2(lo, c, true));
    bfly8(v, sgn);                                                      // c -> b
    wave_xpose<R>(sb, v, t1_r, t1_w);
#pragma unroll
    for (int k1 = 1; k1 < 8; ++k1) v[k1] = mul(v[k1], W.s1(t, k1, true));
    bfly8(v, sgn);                                                      // k1 -> j
  }
}

// Spectral index held by register r of lane t (of LN) after a forward
// transform.
template <int E, int LN = 64>
__device__ __forceinline__ int spec_pos(int t, int r) {
  if constexpr (E == 8) return (t >> 3) + 8 * (t & 7) + 64 * r;
  else return r + E * brev_ln<LN>(t);
}

// Value of the partner position L - m of register r (lane t holds
// m = spec_pos<E, LN>(t, r)).  Lane exchange only; every lane takes part,
// and the partner is always in the lane's own group of LN lanes.
//   E = 8: m = k1 + 8 c + 64 d (lane c + 8 k1) -> register 7 - d of the lane
//          (7 - c) + 8 (8 - k1) for k1 > 0, (8 - c) for k1 = 0 < c; lane 0
//          keeps its own register (8 - d) mod 8.
//   else:  m = r + E b (b = brev(t)) -> register E - r of lane LN - 1 - t,
//          or, for r = 0, register 0 of lane brev((LN - b) mod LN), passed
//          as the wavefront lane `lane0`.
template <typename R, int E, int LN = 64>
__device__ __forceinline__ cx<R> mirror_val(const cx<R> (&v)[E], int r, int lane0) {
  const int t = threadIdx.x & 63;
  if constexpr (E == 8) {
    static_assert(LN == 64, "the E = 8 transform spans the wavefront");
    const int c = t & 7, k1 = t >> 3;
    const int tp = k1 ? (7 - c) + 8 * (8 - k1) : ((8 - c) & 7);
    const cx<R> o = shfl_c(v[7 - r], tp);
    return t == 0 ? v[(8 - r) & 7] : o;
  } else {
    cx<R> out = mk<R>(0, 0);
#pragma unroll
    for (int q = 0; q < E; ++q) {
      // compile-time register selection: every lane takes the same register
      const int want = (r == 0) ? 0 : E - r;
      if (q == want) out = shfl_c(v[q], r == 0 ? lane0 : t ^ (LN - 1));
    }
    return out;
  }
}

// Staging element access.  Strided tiles: row e holds the columns
// (pitch cols + 1); x tiles: row c holds the elements (pitch len + 1).
template <int XP>
__device__ __forceinline__ int sidx(int c, int e, int pitch) {
  return XP ? c * pitch + e : e * pitch + c;
}

// Phases B and C of a pass: the block's staged tile (LDS, after a barrier)
// -> pencil registers, transform(s) (and the Green operator in the fused z
// pass), -> output staging.  `w` is the block's pencil held by this lane's
// group of LN lanes and `t` the lane within that group.  Returns the output
// rows per column; the caller places the barrier before the output staging
// is read.
template <typename R, int MODE, int XP, int E, int LN, typename WP, typename GZ>
__device__ __forceinline__ int wave_pencil(const PassDesc& d, int kind, int n, bool packed, bool half, int cols,
                                           int w, int t, int mlane0, const Tile& tl, int j0, int pitch, R* sr,
                                           cx<R>* sc, R* wscr, WP W, const LaneTw<R, LN>& ltw, const GreenCol<R>* gcol,
                                           GZ gz) {
  constexpr int L = LN * E;
  static_assert(LN == 64 || E != 8, "the E = 8 transform spans the wavefront");
  // ---------------- phase B: pencil -> registers, FFT ----------------
  cx<R> v[E];
  const int ca = packed ? 2 * w : w, cb = 2 * w + 1;   // columns of this pencil
  if (MODE == 0 || MODE == 2) {
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int x = t + LN * j;
      int jn, sg;
      ext_src(kind, n, x, jn, sg);
      cx<R> z = mk<R>(0, 0);
      if (sg) {
        const int e = jn - j0;
        if (packed) z = mk<R>(sr[sidx<XP>(ca, e, pitch)], sr[sidx<XP>(cb, e, pitch)]);
        else z = sc[sidx<XP>(ca, e, pitch)];
        if (sg < 0) z = scl(z, (R)-1);
      }
      v[j] = z;
    }
    if constexpr (E == 8) wave_fft8<R>(v, W, wscr, false);
    else wave_fft<R, E, LN>(v, gconst((const cx<R>*)d.tw), ltw, false);
  } else {
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int m = spec_pos<E, LN>(t, j);   // inverse input layout: lane t, register j
      cx<R> z = mk<R>(0, 0);
      if (half) {
        // two Hermitian half spectra A (column ca) and B (column cb): Z = A + i B
        const int km = m <= n / 2 ? m : n - m;
        cx<R> A = sc[sidx<XP>(ca, km, pitch)], Bv = sc[sidx<XP>(cb, km, pitch)];
        if (m > n / 2) { A = conj(A); Bv = conj(Bv); }
        z = mk<R>(A.re - Bv.im, A.im + Bv.re);
      } else {
        int k;
        R fr, fi;
        if (spec_src<R>(kind, n, m, k, fr, fi)) {
          const cx<R> g = packed ? mk<R>(sr[sidx<XP>(ca, k, pitch)], sr[sidx<XP>(cb, k, pitch)])
                                 : sc[sidx<XP>(ca, k, pitch)];
          z = mul(g, mk<R>(fr, fi));
        }
      }
      v[j] = z;
    }
    if constexpr (E == 8) wave_fft8<R>(v, W, wscr, true);
    else wave_fft<R, E, LN>(v, gconst((const cx<R>*)d.tw), ltw, true);
  }

  if (MODE == 2) {
    // Green operator on the spectrum held in registers (lane t, register k1:
    // position m = spec_pos(t, k1)); same structure-preserving scaling as the
    // generic pass.
    const bool okA = ca < tl.ncol, okB = packed ? cb < tl.ncol : false;
    if (half) {
      cx<R> nv[E];
#pragma unroll
      for (int k1 = 0; k1 < E; ++k1) {
        const int m = spec_pos<E, LN>(t, k1);
        const cx<R> a = v[k1], b = conj(mirror_val<R, E, LN>(v, k1, mlane0));
        const cx<R> A = scl(add(a, b), (R)0.5);
        const cx<R> Bv = mk<R>((R)0.5 * (a.im - b.im), (R)-0.5 * (a.re - b.re));
        const int mk_ = m <= n / 2 ? m : n - m;
        const cx<R> sc2 = gz(mk_);
        const R s2 = sc2.re, c2 = sc2.im;
        const R fa = okA ? green_apply<R>(gcol[ca], s2, c2) : (R)0;
        const R fb = okB ? green_apply<R>(gcol[cb], s2, c2) : (R)0;
        nv[k1] = mk<R>(fa * A.re - fb * Bv.im, fa * A.im + fb * Bv.re);
      }
#pragma unroll
      for (int k1 = 0; k1 < E; ++k1) v[k1] = nv[k1];
    } else {
#pragma unroll
      for (int k1 = 0; k1 < E; ++k1) {
        const int m = spec_pos<E, LN>(t, k1);
        int k;
        R fr, fi;
        if (!spec_src<R>(kind, n, m, k, fr, fi)) { v[k1] = mk<R>(0, 0); continue; }
        const cx<R> sc2 = gz(k);
        const R s2 = sc2.re, c2 = sc2.im;
        if (packed) {
          const R fa = okA ? green_apply<R>(gcol[ca], s2, c2) : (R)0;
          const R fb = okB ? green_apply<R>(gcol[cb], s2, c2) : (R)0;
          v[k1] = (fi == (R)0) ? mk<R>(v[k1].re * fa, v[k1].im * fb) : mk<R>(v[k1].re * fb, v[k1].im * fa);
        } else {
          const R g = okA ? green_apply<R>(gcol[ca], s2, c2) : (R)0;
          v[k1] = scl(v[k1], g);
        }
      }
    }
    if constexpr (E == 8) wave_fft8<R>(v, W, wscr, true);
    else wave_fft<R, E, LN>(v, gconst((const cx<R>*)d.tw), ltw, true);
  }

  // ---------------- phase C: registers -> staging ----------------
  __syncthreads();     // every wavefront has finished reading its inputs
  int outcnt;
  if (MODE == 0) {
    const int M = half ? n / 2 + 1 : n_freq(kind, n);
    outcnt = M;
    const int opitch = XP ? M + 1 : cols + 1;
#pragma unroll
    for (int k1 = 0; k1 < E; ++k1) {
      const int m = spec_pos<E, LN>(t, k1);
      // coefficient index carried by position m (inverse of the Table 1 map)
      int k = -1;
      R fr = 1, fi = 0;
      switch (kind) {
        case K_DFT: if (m < M) k = m; break;
        case K_DCT1: if (m <= n) k = m; break;
        case K_DST1: if (m >= 1 && m <= n - 1) { k = m - 1; fr = 0; fi = 1; } break;
        case K_DCT3: if ((m & 1) && m < 2 * n) { k = (m - 1) >> 1; fr = (R)0.5; } break;
        default: if ((m & 1) && m < 2 * n) { k = (m - 1) >> 1; fr = 0; fi = (R)0.5; } break;
      }
      cx<R> pm = mk<R>(0, 0);
      if (half) pm = conj(mirror_val<R, E, LN>(v, k1, mlane0));    // shuffles: all lanes take part
      if (k < 0) continue;
      if (half) {
        const cx<R> a = v[k1];
        sc[sidx<XP>(ca, k, opitch)] = scl(add(a, pm), (R)0.5);
        sc[sidx<XP>(cb, k, opitch)] = mk<R>((R)0.5 * (a.im - pm.im), (R)-0.5 * (a.re - pm.re));
      } else {
        const cx<R> g = mul(v[k1], mk<R>(fr, fi));
        if (packed) { sr[sidx<XP>(ca, k, opitch)] = g.re; sr[sidx<XP>(cb, k, opitch)] = g.im; }
        else sc[sidx<XP>(ca, k, opitch)] = g;
      }
    }
  } else {
    outcnt = n + 1;
    const int opitch = XP ? n + 2 : cols + 1;
    const R invL = (R)1 / (R)L;
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int x = t + LN * j;
      // node j_node = x for x <= n; the periodic node n copies position 0
      if (x > n) continue;
      const int node = x;
      const int srcx = node_src(kind, n, node);
      cx<R> z = srcx < 0 ? mk<R>(0, 0) : scl(v[j], invL);
      if (kind == K_DFT && x == n) z = mk<R>(0, 0);    // filled below from position 0
      if (packed) { sr[sidx<XP>(ca, node, opitch)] = z.re; sr[sidx<XP>(cb, node, opitch)] = z.im; }
      else sc[sidx<XP>(ca, node, opitch)] = z;
      if (kind == K_DFT && x == 0) {
        if (packed) { sr[sidx<XP>(ca, n, opitch)] = z.re; sr[sidx<XP>(cb, n, opitch)] = z.im; }
        else sc[sidx<XP>(ca, n, opitch)] = z;
      }
    }
  }
  return outcnt;
}

// Phase D of the x passes: output staging -> memory.  Forward: the
// coefficient rows; inverse: u^f += w - sum_k beta_k delta_k and the new
// increment into the ring (FP64 accumulator).  RW: rows per wavefront (the
// tile's rows / 8).
template <typename R, int MODE, int UD, int UX, int RW = 2>
__device__ __forceinline__ void wave_store_x(const PassDesc& d, const FM_GLOBAL Ctrl* C, const Tile& tl,
                                             int64_t out_blk, int outcnt, bool cout_, uint32_t eso, const R* sr,
                                             const cx<R>* sc, int w, int t) {
  const int opitch = outcnt + 1;
  const int s1 = (int)d.out_s1;
  if (MODE == 0) {
    FM_GLOBAL char* gout = (FM_GLOBAL char*)gmut((char*)d.out) + out_blk * (int64_t)eso;
    for (int c = w; c < tl.ncol; c += WAVE_PENCILS) {
      const uint32_t rowe = (uint32_t)(c * s1);
      for (int eb = t; eb < outcnt; eb += UD * 64) {
        if (cout_) {
          cx<R> tv[UD];
#pragma unroll
          for (int u = 0; u < UD; ++u)
            if (eb + 64 * u < outcnt) tv[u] = sc[sidx<1>(c, eb + 64 * u, opitch)];
#pragma unroll
          for (int u = 0; u < UD; ++u)
            if (eb + 64 * u < outcnt) gstc<R>(gout, (rowe + (uint32_t)(eb + 64 * u)) * eso, tv[u]);
        } else {
          R tv[UD];
#pragma unroll
          for (int u = 0; u < UD; ++u)
            if (eb + 64 * u < outcnt) tv[u] = sr[sidx<1>(c, eb + 64 * u, opitch)];
#pragma unroll
          for (int u = 0; u < UD; ++u)
            if (eb + 64 * u < outcnt) gst<R>(gout, (rowe + (uint32_t)(eb + 64 * u)) * eso, tv[u]);
        }
      }
    }
  } else {
    // x inverse: u^f += w - sum_k beta_k delta_k, new increment into the ring
    const int nb = C->n_b;
    R be[MAX_DEPTH];
    const FM_GLOBAL char* dsrc[MAX_DEPTH];
    const FM_GLOBAL char* ring = (const FM_GLOBAL char*)gconst((const R*)d.ring);
#pragma unroll
    for (int q = 0; q < MAX_DEPTH; ++q) {
      be[q] = q < nb ? (R)C->beta[q] : (R)0;
      dsrc[q] = ring + ((int64_t)(q < nb ? C->slot_b[q] : 0) * d.ring_stride + out_blk) * (int64_t)sizeof(R);
    }
    FM_GLOBAL char* dw = (FM_GLOBAL char*)gmut((R*)d.ring) +
                         ((int64_t)C->slot_w * d.ring_stride + out_blk) * (int64_t)sizeof(R);
    FM_GLOBAL char* guf = (FM_GLOBAL char*)gmut(d.uf) + out_blk * (int64_t)sizeof(double);
    // all rows of this wavefront: all loads first, then the stores
    for (int eb = t; eb < outcnt; eb += UX * 64) {
      R dl[RW][UX];
      double uo[RW][UX];
#pragma unroll
      for (int r = 0; r < RW; ++r) {
        const int c = w + WAVE_PENCILS * r;
        const uint32_t rowe = (uint32_t)(c * s1);
#pragma unroll
        for (int u = 0; u < UX; ++u) {
          const int e = eb + 64 * u;
          if (c < tl.ncol && e < outcnt) {
            const uint32_t o = rowe + (uint32_t)e;
            R a = sr[sidx<1>(c, e, opitch)];
#pragma unroll
            for (int q = 0; q < MAX_DEPTH; ++q)
              if (q < nb) a -= be[q] * gld<R>(dsrc[q], o * (uint32_t)sizeof(R));
            dl[r][u] = a;
            uo[r][u] = gld<double>(guf, o * 8u);
          }
        }
      }
#pragma unroll
      for (int r = 0; r < RW; ++r) {
        const int c = w + WAVE_PENCILS * r;
        const uint32_t rowe = (uint32_t)(c * s1);
#pragma unroll
        for (int u = 0; u < UX; ++u) {
          const int e = eb + 64 * u;
          if (c < tl.ncol && e < outcnt) {
            const uint32_t o = rowe + (uint32_t)e;
            gst<R>(dw, o * (uint32_t)sizeof(R), dl[r][u]);
            gst<double>(guf, o * 8u, uo[r][u] + (double)dl[r][u]);
          }
        }
      }
    }
  }
}

// KIND >= 0 fixes the transform kind and PK the packing (1: two real
// columns per pencil, 0: one complex column) at compile time, and with them
// the axis length (n = L / S_f), the tile width, the element types and every
// staging pitch; KIND = -1 reads them from the descriptor.  Global accesses
// use 32-bit byte offsets from a per-block base: the plan keeps each
// component's buffers below 4 GiB for these kernels.  LN < 64 gives every
// group of LN lanes a pencil of its own (L = LN E; the block's tile is
// 64 / LN times wider).
template <typename R, int MODE, int XP, int E, int KIND = -1, int PK = -1, int LN = 64>
__global__ void __launch_bounds__(WAVE_THREADS) k_wave(const PassDesc* __restrict__ descs,
                                                       const int2* __restrict__ work,
                                                       const SolveDev* __restrict__ S) {
  static_assert(LN == 64 || LN == 32 || LN == 16, "lanes per pencil");
  constexpr int NPW = 64 / LN;                    // pencils per wavefront
  constexpr int PPB = WAVE_PENCILS * NPW;         // pencils per block
  constexpr int LPPB = 9 - lanes_log2(LN);        // log2 PPB
  extern __shared__ __align__(16) char smem[];
  __shared__ GreenCol<R> gcol[2 * PPB];
  const int2 wk = work[blockIdx.x];
  const PassDesc& d = descs[wk.x];
  const FM_GLOBAL Ctrl* C = gconst(S[d.solve].ctrl);
  // Only the x forward pass needs the control block to address its inputs
  // (Anderson weights and slots); the others issue their tile loads first
  // and test the solve's status after them, so that the dependent loads of
  // descriptor, control pointer and status do not delay the data.  A stopped
  // solve's buffers stay allocated, and nothing is written for it.
  constexpr bool CTRL_FIRST = MODE == 0 && XP;
  if (CTRL_FIRST && C->status != ST_RUNNING) return;
  constexpr int L = LN * E;
  constexpr bool SK = KIND >= 0;
  // rows loaded by the strided passes when the kind is fixed, and the
  // loads per thread that cover them in one batch
  constexpr int NC = SK ? L / kind_sf(KIND) : 0;
  constexpr int CNT_IN = !SK ? 0
                         : (MODE == 1 && PK == 1 && KIND == K_DFT) ? NC / 2 + 1
                         : KIND == K_DCT1 ? NC + 1 : KIND == K_DST1 ? NC - 1 : NC;
  constexpr int CNT_OUT = !SK ? 0 : MODE != 0 ? NC + 1 : (PK == 1 && KIND == K_DFT) ? NC / 2 + 1
                          : KIND == K_DCT1 ? NC + 1 : KIND == K_DST1 ? NC - 1 : NC;
  constexpr int STEP_C = WAVE_THREADS / (PK == 1 ? 2 * PPB : PPB);
  const int kind = SK ? KIND : d.kind;
  const int n = SK ? L / kind_sf(KIND) : d.n;
  const bool packed = SK ? PK == 1 : d.packed != 0;
  const int lcols = packed ? LPPB + 1 : LPPB;   // tile width: 2 PPB real or PPB complex columns
  const int cols = 1 << lcols;
  const bool half = packed && kind == K_DFT;
  // complex elements in and out (real DTT data travels packed as reals)
  const bool cin = SK ? (MODE == 1 ? (PK != 1 || KIND == K_DFT) : PK != 1) : d.cplx_in != 0;
  const bool cout_ = SK ? (MODE == 0 ? (PK != 1 || KIND == K_DFT) : PK != 1)
                        : (MODE == 0 ? d.cplx_out != 0 : !packed);
  const uint32_t esi = cin ? 2 * sizeof(R) : sizeof(R);
  const uint32_t eso = cout_ ? 2 * sizeof(R) : sizeof(R);
  const int w = threadIdx.x >> 6, t = threadIdx.x & 63;
  const int pen = w * NPW + t / LN, tp = t & (LN - 1);   // this lane's pencil, lane within it
  const int bt = brev_ln<LN>(tp);               // spectral lane order
  const int mlane0 = (t & ~(LN - 1)) + brev_ln<LN>((LN - bt) & (LN - 1));   // partner of register 0
  Tile tl;
  if (XP) { tl.p0b = wk.y * cols; tl.p1 = 0; }
  else { tl.p0b = (wk.y % d.tiles_p0) * cols; tl.p1 = wk.y / d.tiles_p0; }
  tl.ncol = min(cols, d.n_p0 - tl.p0b);
  const FM_GLOBAL cx<R>* W = gconst((const cx<R>*)d.tw);
  // first element of the block's tile, in elements of the input / output
  const int64_t in_blk = XP ? (int64_t)tl.p0b * d.in_s1 : (int64_t)tl.p1 * d.in_s1 + tl.p0b;
  const int64_t out_blk = XP ? (int64_t)tl.p0b * d.out_s1 : (int64_t)tl.p1 * d.out_s1 + tl.p0b;
  LaneTw<R, LN> ltw;
  if constexpr (E != 8) ltw = lane_twiddles<R, LN>(W, L);
  // E = 8: per-wave transpose scratch first, then the staging tile
  R* wscr = (R*)smem + (E == 8 ? w * WT_SIZE : 0);
  char* stage = smem + (E == 8 ? WAVE_PENCILS * WT_SIZE * sizeof(R) : 0);
  R* sr = (R*)stage;           // staging, real elements (packed)
  cx<R>* sc = (cx<R>*)stage;   // staging, complex elements

  if (MODE == 2 && threadIdx.x < cols)
    gcol[threadIdx.x] = green_col<R>(d, min(tl.p0b + (int)threadIdx.x, d.n_p0 - 1), tl.p1);

  // ---------------- phase A: tile -> staging (coalesced) ----------------
  int j0 = 0, cnt;
  if (MODE == 1) cnt = SK ? (half ? n / 2 + 1 : n_freq(kind, n)) : d.len_in;
  else raw_range(kind, n, j0, cnt);
  const int pitch = XP ? cnt + 1 : cols + 1;
  {
    // Loads are issued in batches of U per thread before any is written to
    // the staging array, so that U requests per lane are in flight at once.
    constexpr int U = SK && !XP ? (CNT_IN + STEP_C - 1) / STEP_C : 8;
    if (XP) {
      const int s1 = (int)d.in_s1;
      if (MODE == 0) {
        // x forward: Green input x = sum_q alpha_q D_{slot q} (Anderson mix)
        const int nd = C->n_d;
        R al[MAX_DEPTH];
        const FM_GLOBAL char* src[MAX_DEPTH];
#pragma unroll
        for (int q = 0; q < MAX_DEPTH; ++q) {
          al[q] = q < nd ? (R)C->alpha[q] : (R)0;
          src[q] = (const FM_GLOBAL char*)gconst((const R*)d.ring) +
                   ((int64_t)(q < nd ? C->slot_d[q] : 0) * d.ring_stride + in_blk) * (int64_t)sizeof(R);
        }
        for (int c = w; c < cols; c += WAVE_PENCILS) {
          const bool okc = c < tl.ncol;
          const uint32_t rowe = (uint32_t)(c * s1 + j0);
          for (int eb = t; eb < cnt; eb += U * 64) {
            R tv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
              const int e = eb + 64 * u;
              tv[u] = 0;
              if (okc && e < cnt) {
                const uint32_t o = (rowe + (uint32_t)e) * (uint32_t)sizeof(R);
                R a = al[0] * gld<R>(src[0], o);
#pragma unroll
                for (int q = 1; q < MAX_DEPTH; ++q)
                  if (q < nd) a += al[q] * gld<R>(src[q], o);
                tv[u] = a;
              }
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
              if (eb + 64 * u < cnt) sr[sidx<1>(c, eb + 64 * u, pitch)] = tv[u];
          }
        }
      } else {
        const FM_GLOBAL char* gin = (const FM_GLOBAL char*)gconst((const char*)d.in) + in_blk * (int64_t)esi;
        for (int c = w; c < cols; c += WAVE_PENCILS) {
          const bool okc = c < tl.ncol;
          const uint32_t rowe = (uint32_t)(c * s1 + j0);
          for (int eb = t; eb < cnt; eb += U * 64) {
            if (cin) {
              cx<R> tv[U];
#pragma unroll
              for (int u = 0; u < U; ++u) {
                const int e = eb + 64 * u;
                tv[u] = mk<R>(0, 0);
                if (okc && e < cnt) tv[u] = gldc<R>(gin, (rowe + (uint32_t)e) * esi);
              }
#pragma unroll
              for (int u = 0; u < U; ++u)
                if (eb + 64 * u < cnt) sc[sidx<1>(c, eb + 64 * u, pitch)] = tv[u];
            } else {
              R tv[U];
#pragma unroll
              for (int u = 0; u < U; ++u) {
                const int e = eb + 64 * u;
                tv[u] = 0;
                if (okc && e < cnt) tv[u] = gld<R>(gin, (rowe + (uint32_t)e) * esi);
              }
#pragma unroll
              for (int u = 0; u < U; ++u)
                if (eb + 64 * u < cnt) sr[sidx<1>(c, eb + 64 * u, pitch)] = tv[u];
            }
          }
        }
      }
    } else {
      const FM_GLOBAL char* gin = (const FM_GLOBAL char*)gconst((const char*)d.in) + in_blk * (int64_t)esi;
      const int rows_per = 64 >> lcols;          // 4 (packed) or 8 (complex) rows per wavefront
      const int c = t & (cols - 1);
      const int step = WAVE_PENCILS * rows_per;
      const bool okc = c < tl.ncol;
      const int e0 = w * rows_per + (t >> lcols);
      const uint32_t ostep = (uint32_t)step * (uint32_t)d.in_sa * esi;
      uint32_t o = ((uint32_t)c + (uint32_t)(j0 + e0) * (uint32_t)d.in_sa) * esi;
      for (int eb = e0; eb < cnt; eb += U * step, o += U * ostep) {
        if (cin) {
          cx<R> tv[U];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            tv[u] = mk<R>(0, 0);
            if (okc && eb + u * step < cnt) tv[u] = gldc<R>(gin, o + u * ostep);
          }
#pragma unroll
          for (int u = 0; u < U; ++u)
            if (eb + u * step < cnt) sc[sidx<0>(c, eb + u * step, pitch)] = tv[u];
        } else {
          R tv[U];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            tv[u] = 0;
            if (okc && eb + u * step < cnt) tv[u] = gld<R>(gin, o + u * ostep);
          }
#pragma unroll
          for (int u = 0; u < U; ++u)
            if (eb + u * step < cnt) sr[sidx<0>(c, eb + u * step, pitch)] = tv[u];
        }
      }
    }
  }
  __syncthreads();
  if (!CTRL_FIRST && C->status != ST_RUNNING) return;

  // z Green tables: sin^2 and cos^2 of the half modified frequency
  const FM_GLOBAL char* zs2 = (const FM_GLOBAL char*)gconst(d.gs2[2]);
  const FM_GLOBAL char* zc2 = (const FM_GLOBAL char*)gconst(d.gc2[2]);
  auto gz = [&](int k) { return mk<R>((R)gld<double>(zs2, 8u * k), (R)gld<double>(zc2, 8u * k)); };
  const int outcnt = wave_pencil<R, MODE, XP, E, LN>(d, kind, n, packed, half, cols, pen, tp, mlane0, tl, j0, pitch,
                                                    sr, sc, wscr, TwGlobal<R>{W}, ltw, gcol, gz);
  __syncthreads();

  // ---------------- phase D: staging -> memory (coalesced) ----------------
  constexpr int UD = SK && !XP ? (CNT_OUT + STEP_C - 1) / STEP_C : 8;
  if (XP) {
    wave_store_x<R, MODE, UD, SK ? (CNT_OUT + 63) / 64 : 4 / NPW, 2 * NPW>(d, C, tl, out_blk, outcnt, cout_, eso,
                                                                           sr, sc, w, t);
  } else {
    FM_GLOBAL char* gout = (FM_GLOBAL char*)gmut((char*)d.out) + out_blk * (int64_t)eso;
    const int opitch = cols + 1;
    const int rows_per = 64 >> lcols;
    const int step = WAVE_PENCILS * rows_per;
    const int c = t & (cols - 1);
    const int e0 = w * rows_per + (t >> lcols);
    const uint32_t ostep = (uint32_t)step * (uint32_t)d.out_sa * eso;
    uint32_t o = ((uint32_t)c + (uint32_t)e0 * (uint32_t)d.out_sa) * eso;
    if (c < tl.ncol)
      for (int eb = e0; eb < outcnt; eb += UD * step, o += UD * ostep) {
        if (cout_) {
          cx<R> tv[UD];
#pragma unroll
          for (int u = 0; u < UD; ++u)
            if (eb + u * step < outcnt) tv[u] = sc[sidx<0>(c, eb + u * step, opitch)];
#pragma unroll
          for (int u = 0; u < UD; ++u)
            if (eb + u * step < outcnt) gstc<R>(gout, o + u * ostep, tv[u]);
        } else {
          R tv[UD];
#pragma unroll
          for (int u = 0; u < UD; ++u)
            if (eb + u * step < outcnt) tv[u] = sr[sidx<0>(c, eb + u * step, opitch)];
#pragma unroll
          for (int u = 0; u < UD; ++u)
            if (eb + u * step < outcnt) gst<R>(gout, o + u * ostep, tv[u]);
        }
      }
  }
}

// Persistent, software-pipelined form of the strided E = 8 passes (FP32,
// kind and packing fixed).  Block b takes the work items b, b + G, b + 2G,
// ... (G = gridDim.x, a multiple of 8 when there are at least 8 items, so
// that all items of a block run on the XCD the one-item-per-block launch
// would use), and the tile loads of its next item are in flight while the
// current one is transformed.  The twiddles and the z Green table are read
// from LDS inside the transform: the vector-memory counter completes in
// order, so waiting there for a later global load would also wait for the
// prefetch.  LDS: per-wave transpose scratch, twiddles (L), z Green table
// (p_gtab entries), staging.  The single-transform DTT passes are held to
// 64 VGPRs (8 wavefronts per SIMD, four blocks per compute unit).
__host__ __device__ constexpr int p_gtab(int mode, int kind, int packed, int n) {
  return mode != 2 ? 0 : (kind == K_DFT ? (packed ? n / 2 + 1 : n) : (kind == K_DCT1 ? n + 1 : kind == K_DST1 ? n - 1 : n));
}
__host__ __device__ constexpr size_t p_extra_lds(int mode, int kind, int packed) {
  return (size_t)(512 + p_gtab(mode, kind, packed, 512 / kind_sf(kind))) * 2 * sizeof(float);
}

template <int MODE, int KIND, int PK>
__global__ void __launch_bounds__(WAVE_THREADS, (MODE == 2 || KIND == K_DFT) ? 1 : 8) k_wave_p(const PassDesc* __restrict__ descs,
                                                         const int2* __restrict__ work, int nwork,
                                                         const SolveDev* __restrict__ S) {
  typedef float R;
  extern __shared__ __align__(16) char smem[];
  __shared__ GreenCol<R> gcol[2 * WAVE_PENCILS];
  constexpr int E = 8, L = 512;
  constexpr int n = L / kind_sf(KIND);
  constexpr bool packed = PK == 1;
  constexpr int lcols = packed ? 4 : 3, cols = 1 << lcols;
  constexpr bool half = packed && KIND == K_DFT;
  constexpr bool cin = MODE == 1 ? (!packed || KIND == K_DFT) : !packed;
  constexpr bool cout_ = MODE == 0 ? (!packed || KIND == K_DFT) : !packed;
  constexpr uint32_t esi = cin ? 2 * sizeof(R) : sizeof(R);
  constexpr uint32_t eso = cout_ ? 2 * sizeof(R) : sizeof(R);
  // loaded node range (forward and fused passes) or spectral count (inverse)
  constexpr int j0 = (MODE != 1 && (KIND == K_DST1 || KIND == K_DST3)) ? 1 : 0;
  constexpr int nf = KIND == K_DCT1 ? n + 1 : KIND == K_DST1 ? n - 1 : n;
  constexpr int cnt = (MODE == 1 && half) ? n / 2 + 1 : nf;
  constexpr int rows_per = 64 >> lcols, step = WAVE_PENCILS * rows_per;
  constexpr int UI = (cnt + step - 1) / step;
  constexpr int pitch = cols + 1;
  constexpr int GT = p_gtab(MODE, KIND, PK, n);
  static_assert(GT <= WAVE_THREADS, "one Green entry per thread");
  const int w = threadIdx.x >> 6, t = threadIdx.x & 63;
  const int mlane0 = brev6((64 - brev6(t)) & 63);
  const int c = t & (cols - 1), e0 = w * rows_per + (t >> lcols);
  R* wscr = (R*)smem + w * WT_SIZE;
  char* base = smem + WAVE_PENCILS * WT_SIZE * sizeof(R);
  const FM_LDS cx<R>* tw = (const FM_LDS cx<R>*)(cx<R>*)base;
  cx<R>* gtab = (cx<R>*)base + L;
  char* stage = (char*)(gtab + GT);
  R* sr = (R*)stage;
  cx<R>* sc = (cx<R>*)stage;
  if ((int)blockIdx.x >= nwork) return;
  {
    // twiddles of the two stages (the L = 512 table is the same for every item)
    const FM_GLOBAL char* W = (const FM_GLOBAL char*)gconst((const cx<R>*)descs[work[blockIdx.x].x].tw);
    for (int i = threadIdx.x; i < TW8_LDS; i += WAVE_THREADS) {
      const int idx = i < 448 ? (i & 63) * ((i >> 6) + 1) : 8 * ((i - 448) & 7) * (((i - 448) >> 3) + 1);
      ((cx<R>*)base)[i] = gldc<R>(W, (uint32_t)idx * (uint32_t)sizeof(cx<R>));
    }
  }
  typedef typename std::conditional<cin, cx<R>, R>::type LT;
  LT pre[UI];
  cx<R> preg = mk<R>(0, 0);
  auto issue = [&](int item) {
    const int2 wk = work[item];
    const PassDesc& d = descs[wk.x];
    const int p0b = (wk.y % d.tiles_p0) * cols, p1 = wk.y / d.tiles_p0;
    const bool okc = c < d.n_p0 - p0b;
    const FM_GLOBAL char* gin =
        (const FM_GLOBAL char*)gconst((const char*)d.in) + ((int64_t)p1 * d.in_s1 + p0b) * (int64_t)esi;
    const uint32_t ostep = (uint32_t)step * (uint32_t)d.in_sa * esi;
    const uint32_t o = ((uint32_t)c + (uint32_t)(j0 + e0) * (uint32_t)d.in_sa) * esi;
#pragma unroll
    for (int u = 0; u < UI; ++u) {
      if constexpr (cin) {
        pre[u] = mk<R>(0, 0);
        if (okc && e0 + u * step < cnt) pre[u] = gldc<R>(gin, o + u * ostep);
      } else {
        pre[u] = 0;
        if (okc && e0 + u * step < cnt) pre[u] = gld<R>(gin, o + u * ostep);
      }
    }
    if (MODE == 2 && (int)threadIdx.x < GT)
      preg = mk<R>((R)gld<double>((const FM_GLOBAL char*)gconst(d.gs2[2]), 8u * threadIdx.x),
                   (R)gld<double>((const FM_GLOBAL char*)gconst(d.gc2[2]), 8u * threadIdx.x));
  };
  const LaneTw<R> ltw{};
  int item = blockIdx.x;
  issue(item);
  for (; item < nwork; item += gridDim.x) {
    const int2 wk = work[item];
    const PassDesc& d = descs[wk.x];
    Tile tl;
    tl.p0b = (wk.y % d.tiles_p0) * cols;
    tl.p1 = wk.y / d.tiles_p0;
    tl.ncol = min(cols, d.n_p0 - tl.p0b);
    // stage the prefetched tile (and the z Green table)
#pragma unroll
    for (int u = 0; u < UI; ++u)
      if (e0 + u * step < cnt) {
        if constexpr (cin) sc[sidx<0>(c, e0 + u * step, pitch)] = pre[u];
        else sr[sidx<0>(c, e0 + u * step, pitch)] = pre[u];
      }
    if (MODE == 2) {
      if ((int)threadIdx.x < GT) gtab[threadIdx.x] = preg;
      if ((int)threadIdx.x < cols)
        gcol[threadIdx.x] = green_col<R>(d, min(tl.p0b + (int)threadIdx.x, d.n_p0 - 1), tl.p1);
    }
    __syncthreads();
    const bool run = gconst(S[d.solve].ctrl)->status == ST_RUNNING;
    if (item + (int)gridDim.x < nwork) issue(item + gridDim.x);
    if (run) {
      auto gz = [&](int k) { return gtab[k]; };
      const int outcnt = wave_pencil<R, MODE, 0, E, 64>(d, KIND, n, packed, half, cols, w, t, mlane0, tl, j0, pitch,
                                                    sr, sc, wscr, TwLds<R>{tw}, ltw, gcol, gz);
      __syncthreads();
      FM_GLOBAL char* gout = (FM_GLOBAL char*)gmut((char*)d.out) +
                             ((int64_t)tl.p1 * d.out_s1 + tl.p0b) * (int64_t)eso;
      constexpr int UO = ((MODE == 0 ? (half ? n / 2 + 1 : nf) : n + 1) + step - 1) / step;
      const uint32_t ostep = (uint32_t)step * (uint32_t)d.out_sa * eso;
      const uint32_t o = ((uint32_t)c + (uint32_t)e0 * (uint32_t)d.out_sa) * eso;
      if (c < tl.ncol) {
        if constexpr (cout_) {
          cx<R> tv[UO];
#pragma unroll
          for (int u = 0; u < UO; ++u)
            if (e0 + u * step < outcnt) tv[u] = sc[sidx<0>(c, e0 + u * step, pitch)];
#pragma unroll
          for (int u = 0; u < UO; ++u)
            if (e0 + u * step < outcnt) gstc<R>(gout, o + u * ostep, tv[u]);
        } else {
          R tv[UO];
#pragma unroll
          for (int u = 0; u < UO; ++u)
            if (e0 + u * step < outcnt) tv[u] = sr[sidx<0>(c, e0 + u * step, pitch)];
#pragma unroll
          for (int u = 0; u < UO; ++u)
            if (e0 + u * step < outcnt) gst<R>(gout, o + u * ostep, tv[u]);
        }
      }
    }
    __syncthreads();    // staging free for the next item
  }
}

// Persistent, software-pipelined form of the x forward pass of length 512
// (FP32, two real rows per pencil): as k_wave_p, with the rows of the next
// tile prefetched while the current one is transformed.  The prefetch takes
// the first Anderson slot; the other slots of an Anderson iteration are read
// when the tile is staged.  The template also covers the x inverse pass
// (MODE 1), which the engine keeps on k_wave: measured slower pipelined.
__host__ __device__ constexpr size_t px_extra_lds() { return (size_t)512 * 2 * sizeof(float); }

template <int MODE, int KIND>
__global__ void __launch_bounds__(WAVE_THREADS, (KIND == K_DFT || MODE == 1) ? 1 : 8) k_wave_px(const PassDesc* __restrict__ descs,
                                                                              const int2* __restrict__ work, int nwork,
                                                                              const SolveDev* __restrict__ S) {
  typedef float R;
  extern __shared__ __align__(16) char smem[];
  constexpr int E = 8, L = 512;
  constexpr int n = L / kind_sf(KIND);
  constexpr bool packed = true, half = KIND == K_DFT;
  constexpr int cols = 2 * WAVE_PENCILS;
  constexpr bool cin = MODE == 1 && half;
  constexpr bool cout_ = MODE == 0 && half;
  constexpr uint32_t esi = cin ? 2 * sizeof(R) : sizeof(R);
  constexpr uint32_t eso = cout_ ? 2 * sizeof(R) : sizeof(R);
  constexpr int j0 = (MODE == 0 && (KIND == K_DST1 || KIND == K_DST3)) ? 1 : 0;
  constexpr int nf = KIND == K_DCT1 ? n + 1 : KIND == K_DST1 ? n - 1 : n;
  constexpr int cnt = (MODE == 1 && half) ? n / 2 + 1 : nf;
  constexpr int U1 = (cnt + 63) / 64;
  constexpr int pitch = cnt + 1;
  const int w = threadIdx.x >> 6, t = threadIdx.x & 63;
  const int mlane0 = brev6((64 - brev6(t)) & 63);
  R* wscr = (R*)smem + w * WT_SIZE;
  char* base = smem + WAVE_PENCILS * WT_SIZE * sizeof(R);
  const FM_LDS cx<R>* tw = (const FM_LDS cx<R>*)(cx<R>*)base;
  char* stage = (char*)((cx<R>*)base + L);
  R* sr = (R*)stage;
  cx<R>* sc = (cx<R>*)stage;
  if ((int)blockIdx.x >= nwork) return;
  {
    const FM_GLOBAL char* W = (const FM_GLOBAL char*)gconst((const cx<R>*)descs[work[blockIdx.x].x].tw);
    for (int i = threadIdx.x; i < TW8_LDS; i += WAVE_THREADS) {
      const int idx = i < 448 ? (i & 63) * ((i >> 6) + 1) : 8 * ((i - 448) & 7) * (((i - 448) >> 3) + 1);
      ((cx<R>*)base)[i] = gldc<R>(W, (uint32_t)idx * (uint32_t)sizeof(cx<R>));
    }
  }
  typedef typename std::conditional<cin, cx<R>, R>::type LT;
  LT pre[2][U1];
  // rows of a tile's input: first Anderson slot (forward) or the spectrum (inverse)
  auto row_base = [&](const PassDesc& d, int p0b) -> const FM_GLOBAL char* {
    if (MODE == 0) {
      const FM_GLOBAL Ctrl* C = gconst(S[d.solve].ctrl);
      return (const FM_GLOBAL char*)gconst((const R*)d.ring) +
             ((int64_t)C->slot_d[0] * d.ring_stride + (int64_t)p0b * d.in_s1) * (int64_t)sizeof(R);
    }
    return (const FM_GLOBAL char*)gconst((const char*)d.in) + (int64_t)p0b * d.in_s1 * (int64_t)esi;
  };
  auto issue = [&](int item) {
    const int2 wk = work[item];
    const PassDesc& d = descs[wk.x];
    const int p0b = wk.y * cols;
    const int ncol = d.n_p0 - p0b;
    const FM_GLOBAL char* gin = row_base(d, p0b);
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int c = w + WAVE_PENCILS * r;
      const uint32_t rowe = (uint32_t)(c * (int)d.in_s1 + j0);
#pragma unroll
      for (int u = 0; u < U1; ++u) {
        const int e = t + 64 * u;
        if constexpr (cin) {
          pre[r][u] = mk<R>(0, 0);
          if (c < ncol && e < cnt) pre[r][u] = gldc<R>(gin, (rowe + (uint32_t)e) * esi);
        } else {
          pre[r][u] = 0;
          if (c < ncol && e < cnt) pre[r][u] = gld<R>(gin, (rowe + (uint32_t)e) * esi);
        }
      }
    }
  };
  const LaneTw<R> ltw{};
  const GreenCol<R>* nogreen = nullptr;
  auto nogz = [](int) { return mk<R>(0, 0); };
  int item = blockIdx.x;
  issue(item);
  for (; item < nwork; item += gridDim.x) {
    const int2 wk = work[item];
    const PassDesc& d = descs[wk.x];
    const FM_GLOBAL Ctrl* C = gconst(S[d.solve].ctrl);
    Tile tl;
    tl.p0b = wk.y * cols;
    tl.p1 = 0;
    tl.ncol = min(cols, d.n_p0 - tl.p0b);
    // stage the prefetched rows; an Anderson iteration adds its other slots
    const int nd = MODE == 0 ? C->n_d : 1;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int c = w + WAVE_PENCILS * r;
      if constexpr (MODE == 0) {
        const R a0 = (R)C->alpha[0];
        R v[U1];
#pragma unroll
        for (int u = 0; u < U1; ++u) v[u] = a0 * pre[r][u];
        if (nd > 1 && c < tl.ncol) {
          const uint32_t rowe = (uint32_t)(c * (int)d.in_s1 + j0);
          for (int q = 1; q < nd; ++q) {
            const R aq = (R)C->alpha[q];
            const FM_GLOBAL char* src = (const FM_GLOBAL char*)gconst((const R*)d.ring) +
                                        ((int64_t)C->slot_d[q] * d.ring_stride + (int64_t)tl.p0b * d.in_s1) *
                                            (int64_t)sizeof(R);
#pragma unroll
            for (int u = 0; u < U1; ++u)
              if (t + 64 * u < cnt) v[u] += aq * gld<R>(src, (rowe + (uint32_t)(t + 64 * u)) * (uint32_t)sizeof(R));
          }
        }
#pragma unroll
        for (int u = 0; u < U1; ++u)
          if (t + 64 * u < cnt) sr[sidx<1>(c, t + 64 * u, pitch)] = v[u];
      } else {
#pragma unroll
        for (int u = 0; u < U1; ++u)
          if (t + 64 * u < cnt) {
            if constexpr (cin) sc[sidx<1>(c, t + 64 * u, pitch)] = pre[r][u];
            else sr[sidx<1>(c, t + 64 * u, pitch)] = pre[r][u];
          }
      }
    }
    __syncthreads();
    const bool run = C->status == ST_RUNNING;
    if (item + (int)gridDim.x < nwork) issue(item + gridDim.x);
    if (run) {
      const int outcnt = wave_pencil<R, MODE, 1, E, 64>(d, KIND, n, packed, half, cols, w, t, mlane0, tl, j0, pitch,
                                                    sr, sc, wscr, TwLds<R>{tw}, ltw, nogreen, nogz);
      __syncthreads();
      wave_store_x<R, MODE, 8, (n + 1 + 63) / 64>(d, C, tl, (int64_t)tl.p0b * d.out_s1, outcnt, cout_, eso, sr, sc, w, t);
    }
    __syncthreads();    // staging free for the next item
  }
}

}  // namespace fm

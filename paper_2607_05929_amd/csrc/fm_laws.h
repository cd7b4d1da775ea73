// Behaviour laws evaluated at one integration point (small strain).
// Strain / stress in Voigt order xx yy zz yz xz xy (tensor shears); the
// anisotropic laws work in Mandel form (sqrt 2 on the shears).
//
// Material table entry (MT_STRIDE reals):
//   ISO   : lambda, mu
//   ANISO : C_M (6x6 Mandel stiffness, rotated cubic), upper triangle packed
//           row by row (21 reals)
//   J2    : lambda, mu, sy0, H
//   CP    : rotation R (9, row-major, sample = R crystal) | crystal-frame
//           cubic Mandel stiffness c11, c12, c44m = 2 C44 | compliance s11,
//           s12, s44m = 1 / (2 C44) | gdot0, n, tau0, taus, theta0
// Internal variables (7): plastic strain (Voigt, tensor shears) and the
// cumulated plastic strain p (J2) or accumulated slip Gamma (CP).
#pragma once
#include "fm_common.h"

namespace fm {

enum Law : int { LAW_ISO = 0, LAW_ANISO = 1, LAW_J2 = 2, LAW_CP = 3, LAW_SVK = 4, LAW_NEOHOOKE = 5 };

template <typename R> struct LawTol;
template <> struct LawTol<float> { static constexpr float cp = 2e-6f; };
template <> struct LawTol<double> { static constexpr double cp = 1e-11; };

template <typename R>
__device__ __forceinline__ void to_mandel(const R e[6], R m[6]) {
  const R s2 = (R)1.41421356237309504880;
  m[0] = e[0]; m[1] = e[1]; m[2] = e[2]; m[3] = s2 * e[3]; m[4] = s2 * e[4]; m[5] = s2 * e[5];
}
template <typename R>
__device__ __forceinline__ void from_mandel(const R m[6], R e[6]) {
  const R is2 = (R)0.70710678118654752440;
  e[0] = m[0]; e[1] = m[1]; e[2] = m[2]; e[3] = is2 * m[3]; e[4] = is2 * m[4]; e[5] = is2 * m[5];
}

template <typename R, typename PT>
__device__ __forceinline__ void mat6(PT M, const R x[6], R y[6]) {
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    R a = 0;
#pragma unroll
    for (int j = 0; j < 6; ++j) a += M[i * 6 + j] * x[j];
    y[i] = a;
  }
}

// y = C x for a symmetric 6x6 matrix stored as its packed upper triangle.
template <typename R, typename PT>
__device__ __forceinline__ void mat6sym(PT Cp, const R x[6], R y[6]) {
  R c[21];
#pragma unroll
  for (int k = 0; k < 21; ++k) c[k] = Cp[k];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    R a = 0;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const int lo = i < j ? i : j, hi = i < j ? j : i;
      a += c[lo * 6 - lo * (lo - 1) / 2 + (hi - lo)] * x[j];
    }
    y[i] = a;
  }
}

// |r|^n: binary powering for integral exponents up to 64 (the usual rate
// sensitivities), exp(n log |r|) otherwise.
template <typename R>
__device__ __forceinline__ R powabs(R r, R n) {
  const R a = r < 0 ? -r : r;
  if (a == (R)0) return (R)0;
  if (n >= (R)0 && n <= (R)64 && n == floor(n)) {
    int k = (int)n;
    R base = a, acc = 1;
    while (k) {
      if (k & 1) acc *= base;
      base *= base;
      k >>= 1;
    }
    return acc;
  }
  return exp(n * log(a));
}

// FCC {111}<110> slip systems in the crystal frame (unnormalised slip
// direction m and plane normal n, |m| = sqrt 2, |n| = sqrt 3).
constexpr int FCC_M[12][3] = {{1, -1, 0}, {1, 0, -1}, {0, 1, -1}, {1, 1, 0}, {1, 0, 1},  {0, 1, -1},
                              {1, 1, 0},  {1, 0, -1}, {0, 1, 1},  {1, -1, 0}, {1, 0, 1}, {0, 1, 1}};
constexpr int FCC_N[12][3] = {{1, 1, 1},  {1, 1, 1},  {1, 1, 1},  {-1, 1, 1}, {-1, 1, 1}, {-1, 1, 1},
                              {1, -1, 1}, {1, -1, 1}, {1, -1, 1}, {1, 1, -1}, {1, 1, -1}, {1, 1, -1}};
constexpr int MND_I[6] = {0, 1, 2, 1, 0, 0}, MND_J[6] = {0, 1, 2, 2, 2, 1};

// Mandel component a of the Schmid tensor sym(m (x) n) / (|m| |n|) of
// system s (both compile-time after unrolling: the values fold to literals).
template <typename R>
__device__ __forceinline__ R schmid_c(int s, int a) {
  const int i = MND_I[a], j = MND_J[a];
  const int v2 = FCC_M[s][i] * FCC_N[s][j] + FCC_M[s][j] * FCC_N[s][i];   // 2 sym(m n)_ij
  const double f = 0.5 / (1.41421356237309504880 * 1.73205080756887729353);
  return (R)(a < 3 ? v2 * f : v2 * f * 1.41421356237309504880);
}

// Rotation of a symmetric tensor in Mandel form: to the crystal frame
// (R^T A R) or back to the sample frame (R A R^T).
template <typename R>
__device__ __forceinline__ void mandel_rotate(const R (&Rm)[3][3], const R a[6], R b[6], bool to_crystal) {
  const R is2 = (R)0.70710678118654752440, s2 = (R)1.41421356237309504880;
  const R A[3][3] = {{a[0], is2 * a[5], is2 * a[4]}, {is2 * a[5], a[1], is2 * a[3]}, {is2 * a[4], is2 * a[3], a[2]}};
  R T[3][3], B[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      R t = 0;
#pragma unroll
      for (int k = 0; k < 3; ++k) t += A[i][k] * (to_crystal ? Rm[k][j] : Rm[j][k]);
      T[i][j] = t;
    }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j) {
      R t = 0;
#pragma unroll
      for (int k = 0; k < 3; ++k) t += (to_crystal ? Rm[k][i] : Rm[i][k]) * T[k][j];
      B[i][j] = t;
    }
  b[0] = B[0][0]; b[1] = B[1][1]; b[2] = B[2][2];
  b[3] = s2 * B[1][2]; b[4] = s2 * B[0][2]; b[5] = s2 * B[0][1];
}

// Backward-Euler FCC crystal viscoplasticity, solved in the crystal frame
// (the equations are invariant under the rotation; there the Schmid tensors
// are constants and the cubic compliance has three entries): Newton on
// sigma_M, dGamma with backtracking, started from the elastic predictor
// scaled to |tau|/tau_c <= 2, or from the stress sp of the point's previous
// evaluation (Mandel, sample frame; with the slip its rates give at the
// increment's initial hardness) when that has the smaller residual: within
// an increment the strain changes little between iterations, so the
// previous stress is a few Newton steps closer to the solution.  Stops at
// the tolerance or when no backtracked step lowers the residual.
template <typename R, typename PT>
__device__ void cp_update(PT P, const R em[6], const R epn[6], R Gn, R dt, R sm[6], R epm[6], R& Gout,
                          const R* sp = nullptr) {
  R Rm[3][3];
#pragma unroll
  for (int i = 0; i < 9; ++i) Rm[i / 3][i % 3] = P[i];
  const R c11 = P[9], c12 = P[10], c44 = P[11], s11 = P[12], s12 = P[13], s44 = P[14];
  const R g0 = P[15], nx = P[16], tau0 = P[17], taus = P[18], th0 = P[19];
  R ee[6];
  {
    R es[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) es[i] = em[i] - epn[i];
    mandel_rotate<R>(Rm, es, ee, true);
  }
  R escale = (R)1e-9;
#pragma unroll
  for (int i = 0; i < 6; ++i) escale = fmax(escale, fabs(ee[i]));
  auto comp = [&](const R* x, R* y) {       // crystal-frame compliance
    y[0] = s11 * x[0] + s12 * (x[1] + x[2]);
    y[1] = s11 * x[1] + s12 * (x[0] + x[2]);
    y[2] = s11 * x[2] + s12 * (x[0] + x[1]);
    y[3] = s44 * x[3]; y[4] = s44 * x[4]; y[5] = s44 * x[5];
  };
  auto tau_of = [&](const R* sg, int s_) {
    R t = 0;
#pragma unroll
    for (int i = 0; i < 6; ++i) t += sg[i] * schmid_c<R>(s_, i);
    return t;
  };
  R sig[6];
  sig[0] = c11 * ee[0] + c12 * (ee[1] + ee[2]);
  sig[1] = c11 * ee[1] + c12 * (ee[0] + ee[2]);
  sig[2] = c11 * ee[2] + c12 * (ee[0] + ee[1]);
  sig[3] = c44 * ee[3]; sig[4] = c44 * ee[4]; sig[5] = c44 * ee[5];
  R dG = 0;
  {
    const R tc = tau0 + (taus - tau0) * (1 - exp(-th0 * Gn / (taus - tau0)));
    R rmax = 0;
#pragma unroll
    for (int s_ = 0; s_ < 12; ++s_) rmax = fmax(rmax, fabs(tau_of(sig, s_)));
    rmax /= tc;
    if (rmax > (R)2) {
      const R f = (R)2 / rmax;
#pragma unroll
      for (int i = 0; i < 6; ++i) sig[i] *= f;
    }
  }
  const R ihs = (R)1 / (taus - tau0), iesc = (R)1 / escale;
  // slip rate of system s_ at resolved shear ratio r
  auto rate = [&](R r) { return g0 * powabs(r, nx) * (r < 0 ? (R)-1 : (R)1); };
  auto resid = [&](const R* sg, R d, R* Rs, R& Rg, R& tc) -> R {
    tc = tau0 + (taus - tau0) * (1 - exp(-th0 * (Gn + d) * ihs));
    const R itc = (R)1 / tc;
    R eps_s[6];
    comp(sg, eps_s);
#pragma unroll
    for (int i = 0; i < 6; ++i) Rs[i] = eps_s[i] - ee[i];
    R sum = 0;
#pragma unroll
    for (int s_ = 0; s_ < 12; ++s_) {
      const R g = rate(tau_of(sg, s_) * itc);
      sum += fabs(g);
#pragma unroll
      for (int i = 0; i < 6; ++i) Rs[i] += dt * g * schmid_c<R>(s_, i);
    }
    Rg = d - dt * sum;
    R nr = fabs(Rg);
#pragma unroll
    for (int i = 0; i < 6; ++i) nr = fmax(nr, fabs(Rs[i]));
    return nr * iesc;
  };
  // (the slip rates are recomputed where needed rather than kept: registers)
  R Rs[6], Rg, tc;
  R nr = resid(sig, dG, Rs, Rg, tc);
  if (sp) {
    R sc[6];
    mandel_rotate<R>(Rm, sp, sc, true);
    const R itc0 = (R)1 / (tau0 + (taus - tau0) * (1 - exp(-th0 * Gn * ihs)));
    R d0 = 0;
#pragma unroll
    for (int s_ = 0; s_ < 12; ++s_) d0 += fabs(rate(tau_of(sc, s_) * itc0));
    d0 *= dt;
    R Rs_b[6], Rg_b, tc_b;
    const R nr_b = resid(sc, d0, Rs_b, Rg_b, tc_b);
    if (nr_b < nr) {
#pragma unroll
      for (int i = 0; i < 6; ++i) { sig[i] = sc[i]; Rs[i] = Rs_b[i]; }
      dG = d0; Rg = Rg_b; tc = tc_b; nr = nr_b;
    }
  }
  for (int it = 0; it < 80 && nr >= LawTol<R>::cp; ++it) {
    // Newton matrix [[A, b], [c^T, d6]] on (sigma_M, dGamma): A = compliance +
    // sum_s dt a_s P_s P_s^T is symmetric positive definite, so the step is an
    // L D L^T solve of A against the residual and b, closed by the scalar
    // Schur complement (no pivoting; the lower triangle of A only; six
    // reciprocals of the pivots and no square root or further division)
    const R hG = th0 * exp(-th0 * (Gn + dG) * ihs);
    const R itc = (R)1 / tc;
    R A[6][6], bv[6], cv[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      bv[i] = 0; cv[i] = 0;
#pragma unroll
      for (int j2 = 0; j2 <= i; ++j2) A[i][j2] = 0;
    }
    A[0][0] = s11; A[1][1] = s11; A[2][2] = s11;
    A[1][0] = s12; A[2][0] = s12; A[2][1] = s12;
    A[3][3] = s44; A[4][4] = s44; A[5][5] = s44;
    R d6 = 1;
#pragma unroll
    for (int s_ = 0; s_ < 12; ++s_) {
      const R r = tau_of(sig, s_) * itc;
      const R pw = powabs(r, nx - 1);
      const R a = nx * g0 * pw * itc;
      const R sg = r < 0 ? (R)-1 : (R)1;
      const R gs = g0 * pw * fabs(r) * sg;          // slip rate g0 |r|^n sign r
      const R ca = dt * a, cb = dt * nx * gs * itc * hG, cc = dt * sg * a;
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        const R pi = schmid_c<R>(s_, i);
#pragma unroll
        for (int j2 = 0; j2 <= i; ++j2) A[i][j2] += ca * pi * schmid_c<R>(s_, j2);
        bv[i] -= cb * pi;
        cv[i] -= cc * pi;
      }
      d6 += dt * nx * fabs(gs) * itc * hG;
    }
    // A = L D L^T: unit lower L in the strict lower triangle of A, D in dd,
    // 1 / D in id
    bool spd = true;
    R dd[6], id[6];
#pragma unroll
    for (int j2 = 0; j2 < 6; ++j2) {
      R v[6];
      R dj = A[j2][j2];
#pragma unroll
      for (int k = 0; k < j2; ++k) {
        v[k] = A[j2][k] * dd[k];
        dj -= A[j2][k] * v[k];
      }
      spd = spd && dj > 0;
      dd[j2] = dj;
      id[j2] = (R)1 / fmax(dj, (R)1e-300);
#pragma unroll
      for (int i = j2 + 1; i < 6; ++i) {
        R t = A[i][j2];
#pragma unroll
        for (int k = 0; k < j2; ++k) t -= A[i][k] * v[k];
        A[i][j2] = t * id[j2];
      }
    }
    if (!spd) break;
    // z1 = A^-1 Rs, z2 = A^-1 b (forward substitution, pivots, backward)
    R z1[6], z2[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      R t1 = Rs[i], t2 = bv[i];
#pragma unroll
      for (int k = 0; k < i; ++k) { t1 -= A[i][k] * z1[k]; t2 -= A[i][k] * z2[k]; }
      z1[i] = t1;
      z2[i] = t2;
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) { z1[i] *= id[i]; z2[i] *= id[i]; }
#pragma unroll
    for (int i = 5; i >= 0; --i) {
      R t1 = z1[i], t2 = z2[i];
#pragma unroll
      for (int k = i + 1; k < 6; ++k) { t1 -= A[k][i] * z1[k]; t2 -= A[k][i] * z2[k]; }
      z1[i] = t1;
      z2[i] = t2;
    }
    R cz1 = 0, cz2 = 0;
#pragma unroll
    for (int i = 0; i < 6; ++i) { cz1 += cv[i] * z1[i]; cz2 += cv[i] * z2[i]; }
    R dx[7];
    dx[6] = (Rg - cz1) / (d6 - cz2);
#pragma unroll
    for (int i = 0; i < 6; ++i) dx[i] = z1[i] - z2[i] * dx[6];
    R lam = 1;
    R s_new[6], d_new, Rs2[6], Rg2, tc2, nr2 = nr;
    bool improved = false;
    for (int ls = 0; ls < 30; ++ls) {
#pragma unroll
      for (int i = 0; i < 6; ++i) s_new[i] = sig[i] - lam * dx[i];
      d_new = fmax(dG - lam * dx[6], (R)0);
      nr2 = resid(s_new, d_new, Rs2, Rg2, tc2);
      if (nr2 < nr) { improved = true; break; }
      if (lam < (R)1e-7) break;
      lam *= (R)0.5;
    }
    // No step decreases the residual: the iterate sits at the rounding floor
    // of R; keep it (further Newton steps would only repeat the search).
    if (!improved) break;
#pragma unroll
    for (int i = 0; i < 6; ++i) { sig[i] = s_new[i]; Rs[i] = Rs2[i]; }
    dG = d_new; Rg = Rg2; tc = tc2; nr = nr2;
  }
  // back to the sample frame: stress and plastic strain increment
  R dp[6] = {0, 0, 0, 0, 0, 0};
  {
    const R itc = (R)1 / tc;
#pragma unroll
    for (int s_ = 0; s_ < 12; ++s_) {
      const R g = rate(tau_of(sig, s_) * itc);
#pragma unroll
      for (int i = 0; i < 6; ++i) dp[i] += dt * g * schmid_c<R>(s_, i);
    }
  }
  mandel_rotate<R>(Rm, sig, sm, false);
  R dps[6];
  mandel_rotate<R>(Rm, dp, dps, false);
#pragma unroll
  for (int i = 0; i < 6; ++i) epm[i] = epn[i] + dps[i];
  Gout = Gn + dG;
}

// Elastic laws only (isotropic, rotated anisotropic).
template <typename R, typename PT>
__device__ __forceinline__ void law_elastic(int law, PT P, const R eps[6], R sig[6],
                                            const R st[7], R stn[7]) {
  if (law == LAW_ISO) {
    const R lam = P[0], mu = P[1];
    const R tr = eps[0] + eps[1] + eps[2];
#pragma unroll
    for (int i = 0; i < 3; ++i) sig[i] = 2 * mu * eps[i] + lam * tr;
#pragma unroll
    for (int i = 3; i < 6; ++i) sig[i] = 2 * mu * eps[i];
  } else {
    R em[6], sm[6];
    to_mandel(eps, em);
    mat6sym<R>(P, em, sm);
    from_mandel(sm, sig);
  }
#pragma unroll
  for (int i = 0; i < 7; ++i) stn[i] = st[i];
}

// Elastic laws with engineering shear strains (eps[3..5] twice the tensor
// components), as the fused real-space kernel forms them, from the entry's
// Voigt stiffness c (packed upper triangle, stored at MT_VOIGT; no Mandel
// factors on either side); isotropic entries use lambda = c_12, mu = c_44.
template <typename R, int NP>
__device__ __forceinline__ void law_elastic_pts_eng(int law, const R (&c)[21], const R (&eps)[2][6], R (&sig)[2][6]) {
  if (law == LAW_ISO) {
    const R lam = c[1], mu = c[15], mu2 = mu + mu;
#pragma unroll
    for (int r = 0; r < NP; ++r) {
      const R tr = eps[r][0] + eps[r][1] + eps[r][2];
#pragma unroll
      for (int i = 0; i < 3; ++i) sig[r][i] = mu2 * eps[r][i] + lam * tr;
#pragma unroll
      for (int i = 3; i < 6; ++i) sig[r][i] = mu * eps[r][i];
    }
  } else {
#pragma unroll
    for (int r = 0; r < NP; ++r) mat6sym<R>(c, eps[r], sig[r]);
  }
}

// All-zero material entry (the elastic laws give zero stress on it).
__device__ const float k_zero_material32[MT_VOIGT + 21] = {};
__device__ const double k_zero_material64[MT_VOIGT + 21] = {};
template <typename R>
__device__ __forceinline__ const FM_GLOBAL R* zero_material() {
  if constexpr (sizeof(R) == 4) return (const FM_GLOBAL R*)k_zero_material32;
  else return (const FM_GLOBAL R*)k_zero_material64;
}

// sp: the stress of the point's previous evaluation (Voigt), a start for
// the crystal-plasticity Newton solve, or null.
template <typename R, typename PT>
__device__ __forceinline__ void law_eval(int law, PT P, const R eps[6], R sig[6], const R st[7],
                                         R stn[7], R dt, const R* sp = nullptr) {
  if (law == LAW_ISO) {
    const R lam = P[0], mu = P[1];
    const R tr = eps[0] + eps[1] + eps[2];
#pragma unroll
    for (int i = 0; i < 3; ++i) sig[i] = 2 * mu * eps[i] + lam * tr;
#pragma unroll
    for (int i = 3; i < 6; ++i) sig[i] = 2 * mu * eps[i];
#pragma unroll
    for (int i = 0; i < 7; ++i) stn[i] = st[i];
  } else if (law == LAW_ANISO) {
    R em[6], sm[6];
    to_mandel(eps, em);
    mat6sym<R>(P, em, sm);
    from_mandel(sm, sig);
#pragma unroll
    for (int i = 0; i < 7; ++i) stn[i] = st[i];
  } else if (law == LAW_J2) {
    const R lam = P[0], mu = P[1], sy0 = P[2], H = P[3];
    R ee[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) ee[i] = eps[i] - st[i];
    const R tr = ee[0] + ee[1] + ee[2];
    R s[6];
#pragma unroll
    for (int i = 0; i < 3; ++i) sig[i] = 2 * mu * ee[i] + lam * tr;
#pragma unroll
    for (int i = 3; i < 6; ++i) sig[i] = 2 * mu * ee[i];
    const R pm = (sig[0] + sig[1] + sig[2]) / 3;
#pragma unroll
    for (int i = 0; i < 6; ++i) s[i] = sig[i] - (i < 3 ? pm : (R)0);
    const R ss = s[0] * s[0] + s[1] * s[1] + s[2] * s[2] + 2 * (s[3] * s[3] + s[4] * s[4] + s[5] * s[5]);
    const R q = sqrt((R)1.5 * ss);
    const R f = q - (sy0 + H * st[6]);
#pragma unroll
    for (int i = 0; i < 7; ++i) stn[i] = st[i];
    if (f > 0) {
      const R dp = f / (3 * mu + H);
      const R fac = 1 - 3 * mu * dp / q;
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        sig[i] = (i < 3 ? pm : (R)0) + fac * s[i];
        stn[i] = st[i] + (R)1.5 * dp * s[i] / q;
      }
      stn[6] = st[6] + dp;
    }
  } else {
    R em[6], epn[6], sm[6], epm[6], G, spm[6];
    to_mandel(eps, em);
    to_mandel(st, epn);
    if (sp) to_mandel(sp, spm);
    cp_update<R>(P, em, epn, st[6], dt, sm, epm, G, sp ? spm : nullptr);
    from_mandel(sm, sig);
    from_mandel(epm, stn);
    stn[6] = G;
  }
}

// Plastic laws are evaluated in FP64 from an FP64 strain whatever the
// storage precision (internal variables and the stress are stored in R).
// The flow rule's power law (exponent n = 20 in the FCC workloads) amplifies
// the rounding of a resolved shear n-fold, so an FP32 return mapping only
// reaches ~1e-6 relative accuracy, the size of the equilibrium tolerance; and
// the yield / flow switches of a law fed an FP32 strain flip between
// iterations on its rounding.  Both stall the FP32 solve; in FP64 the stress
// is a smooth function of u^f and the FP32 solve converges as the FP64 one.
template <typename R, typename PT>
__device__ __forceinline__ void law_eval_e64(int law, PT P, const double eps[6], R sig[6], const R st[7], R stn[7],
                                             double dt, const R* sp = nullptr) {
  double s[6], a[7], b[7], spd[6];
#pragma unroll
  for (int i = 0; i < 7; ++i) a[i] = st[i];
  if (sp) {
#pragma unroll
    for (int i = 0; i < 6; ++i) spd[i] = sp[i];
  }
  law_eval<double>(law, P, eps, s, a, b, dt, sp ? spd : nullptr);
#pragma unroll
  for (int i = 0; i < 6; ++i) sig[i] = (R)s[i];
#pragma unroll
  for (int i = 0; i < 7; ++i) stn[i] = (R)b[i];
}

}  // namespace fm

// Behaviour laws evaluated at one integration point (small strain).
// Strain / stress in Voigt order xx yy zz yz xz xy (tensor shears); the
// anisotropic laws work in Mandel form (sqrt 2 on the shears).
//
// Material table entry (MT_STRIDE reals):
//   ISO   : lambda, mu
//   ANISO : C_M (6x6 Mandel stiffness, rotated cubic), upper triangle packed
//           row by row (21 reals)
//   J2    : lambda, mu, sy0, H
//   CP    : C_M (36) | S_M = C_M^-1 (36) | Schmid tensors P_M (12 x 6) |
//           gdot0, n, tau0, taus, theta0
// Internal variables (7): plastic strain (Voigt, tensor shears) and the
// cumulated plastic strain p (J2) or accumulated slip Gamma (CP).
#pragma once
#include "fm_common.h"

namespace fm {

enum Law : int { LAW_ISO = 0, LAW_ANISO = 1, LAW_J2 = 2, LAW_CP = 3 };

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

template <typename R>
__device__ __forceinline__ R powabs(R r, R n) {
  const R a = r < 0 ? -r : r;
  if (a == (R)0) return (R)0;
  return exp(n * log(a));
}

// Backward-Euler FCC crystal viscoplasticity (Newton on sigma_M, dGamma with
// backtracking, started from the elastic predictor scaled to |tau|/tau_c <= 2;
// stops at the tolerance or when no backtracked step lowers the residual).
template <typename R, typename PT>
__device__ void cp_update(PT P, const R em[6], const R epn[6], R Gn, R dt, R sm[6], R epm[6], R& Gout) {
  const PT Cm = P;
  const PT Sm = P + 36;
  const PT Pm = P + 72;
  const R g0 = P[144], nx = P[145], tau0 = P[146], taus = P[147], th0 = P[148];
  R ee[6];
  R escale = (R)1e-9;
#pragma unroll
  for (int i = 0; i < 6; ++i) { ee[i] = em[i] - epn[i]; escale = fmax(escale, fabs(ee[i])); }
  R sig[6];
  mat6(Cm, ee, sig);
  R dG = 0;
  {
    const R tc = tau0 + (taus - tau0) * (1 - exp(-th0 * Gn / (taus - tau0)));
    R rmax = 0;
    for (int s = 0; s < 12; ++s) {
      R t = 0;
#pragma unroll
      for (int i = 0; i < 6; ++i) t += sig[i] * Pm[s * 6 + i];
      rmax = fmax(rmax, fabs(t) / tc);
    }
    if (rmax > (R)2) {
      const R f = (R)2 / rmax;
#pragma unroll
      for (int i = 0; i < 6; ++i) sig[i] *= f;
    }
  }
  auto resid = [&](const R* sg, R d, R* Rs, R& Rg, R* gd, R& tc) -> R {
    tc = tau0 + (taus - tau0) * (1 - exp(-th0 * (Gn + d) / (taus - tau0)));
    R eps_s[6];
    mat6<R>(Sm, sg, eps_s);
#pragma unroll
    for (int i = 0; i < 6; ++i) Rs[i] = eps_s[i] - ee[i];
    R sum = 0;
    for (int s = 0; s < 12; ++s) {
      R t = 0;
#pragma unroll
      for (int i = 0; i < 6; ++i) t += sg[i] * Pm[s * 6 + i];
      const R r = t / tc;
      const R g = g0 * powabs(r, nx) * (r < 0 ? (R)-1 : (R)1);
      gd[s] = g;
      sum += fabs(g);
#pragma unroll
      for (int i = 0; i < 6; ++i) Rs[i] += dt * g * Pm[s * 6 + i];
    }
    Rg = d - dt * sum;
    R nr = fabs(Rg);
#pragma unroll
    for (int i = 0; i < 6; ++i) nr = fmax(nr, fabs(Rs[i]));
    return nr / escale;
  };
  R Rs[6], Rg, gd[12], tc;
  R nr = resid(sig, dG, Rs, Rg, gd, tc);
  for (int it = 0; it < 80 && nr >= LawTol<R>::cp; ++it) {
    R J[7][8];
    const R hG = th0 * exp(-th0 * (Gn + dG) / (taus - tau0));
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
      for (int j = 0; j < 6; ++j) J[i][j] = Sm[i * 6 + j];
#pragma unroll
    for (int i = 0; i < 7; ++i) J[i][6] = 0;
#pragma unroll
    for (int j = 0; j < 6; ++j) J[6][j] = 0;
    J[6][6] = 1;
    for (int s = 0; s < 12; ++s) {
      R t = 0;
#pragma unroll
      for (int i = 0; i < 6; ++i) t += sig[i] * Pm[s * 6 + i];
      const R r = t / tc;
      const R a = nx * g0 * powabs(r, nx - 1) / tc;
      const R sg = r < 0 ? (R)-1 : (R)1;
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        const R pi = Pm[s * 6 + i];
#pragma unroll
        for (int j = 0; j < 6; ++j) J[i][j] += dt * a * pi * Pm[s * 6 + j];
        J[i][6] -= dt * nx * gd[s] / tc * hG * pi;
        J[6][i] -= dt * sg * a * pi;
      }
      J[6][6] += dt * nx * fabs(gd[s]) / tc * hG;
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) J[i][7] = Rs[i];
    J[6][7] = Rg;
    // Gaussian elimination with partial pivoting
    for (int p = 0; p < 7; ++p) {
      int piv = p;
      R best = fabs(J[p][p]);
      for (int q = p + 1; q < 7; ++q) if (fabs(J[q][p]) > best) { best = fabs(J[q][p]); piv = q; }
      if (piv != p)
        for (int c = 0; c < 8; ++c) { const R tmp = J[p][c]; J[p][c] = J[piv][c]; J[piv][c] = tmp; }
      const R ip = (R)1 / J[p][p];
      for (int q = p + 1; q < 7; ++q) {
        const R f = J[q][p] * ip;
        for (int c = p; c < 8; ++c) J[q][c] -= f * J[p][c];
      }
    }
    R dx[7];
    for (int p = 6; p >= 0; --p) {
      R t = J[p][7];
      for (int c = p + 1; c < 7; ++c) t -= J[p][c] * dx[c];
      dx[p] = t / J[p][p];
    }
    R lam = 1;
    R s_new[6], d_new, Rs2[6], Rg2, gd2[12], tc2, nr2 = nr;
    bool improved = false;
    for (int ls = 0; ls < 30; ++ls) {
#pragma unroll
      for (int i = 0; i < 6; ++i) s_new[i] = sig[i] - lam * dx[i];
      d_new = fmax(dG - lam * dx[6], (R)0);
      nr2 = resid(s_new, d_new, Rs2, Rg2, gd2, tc2);
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
    for (int s = 0; s < 12; ++s) gd[s] = gd2[s];
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    sm[i] = sig[i];
    R e = epn[i];
    for (int s = 0; s < 12; ++s) e += dt * gd[s] * Pm[s * 6 + i];
    epm[i] = e;
  }
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

template <typename R, typename PT>
__device__ __forceinline__ void law_eval(int law, PT P, const R eps[6], R sig[6], const R st[7],
                                         R stn[7], R dt) {
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
    R em[6], epn[6], sm[6], epm[6], G;
    to_mandel(eps, em);
    to_mandel(st, epn);
    cp_update<R>(P, em, epn, st[6], dt, sm, epm, G);
    from_mandel(sm, sig);
    from_mandel(epm, stn);
    stn[6] = G;
  }
}

}  // namespace fm

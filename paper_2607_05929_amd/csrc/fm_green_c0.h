// C0 discrete Green operator (Sec. 2.6.1, small-strain form of Appendix A)
// applied per frequency to the three components at once.
//
// Under the normal-mixed conditions of Eq. SGO_BCs the three components
// share, along every axis, one set of physical frequencies: the normal
// component and the tangential ones use opposite transforms (DCT-I / DST-I,
// DCT-III / DST-III, or the DFT for all), whose frequencies coincide, with
// the sine transform of a DCT-I / DST-I pair lacking the frequencies 0 and
// pi (its coefficient there is zero and the coupling to it vanishes).  On
// the virtually extended fields the operator is the periodic one,
//   -p^ = K u^,  K = mu0 |xi|^2 I + (mu0 + lambda0) Re(xi xi^H)
// (HEX1: xi real; TETRA2: xi = xi_T2, complex), and the extended spectrum of
// component q is its transform coefficient times the product of the Table 1
// factors alpha of its kinds.  Along an axis the paired kinds have factors
// of equal modulus, so the components differ by the phases
// phi_q = (-i)^(number of sine transforms of q) only, and in transform space
//   u_q = - conj(phi_q) sum_i (K^-1)_qi phi_i p_i.
// Like the B0 / 2mu0 z pass, the kernel applies minus this operator (the
// update adds IDT(DT(x) K^-1) for the Green input x).
// K is real symmetric positive definite off the null modes (|xi| = 0, set to
// zero as for B0: the sin / cos tables hold exact 0 and 1 at the flagged
// frequencies, so |xi|^2 == 0 is the index rule of R7).
#pragma once
#include "fm_fft.h"

namespace fm {

constexpr int C0_TILE = 256;

template <typename R>
__device__ __forceinline__ cx<R> phase_mul(cx<R> v, int k, bool conj_phase) {
  // v (-i)^k, or v i^k when conj_phase
  k &= 3;
  if (conj_phase) k = (4 - k) & 3;
  switch (k) {
    case 0: return v;
    case 1: return mk<R>(v.im, -v.re);     // -i v
    case 2: return mk<R>(-v.re, -v.im);
    default: return mk<R>(-v.im, v.re);    // i v
  }
}

template <typename R>
__global__ void __launch_bounds__(C0_TILE) k_green_c0(const SolveDev* __restrict__ S, const int2* __restrict__ work) {
  const int2 w = work[blockIdx.x];
  const SolveDev& s = S[w.x];
  const FM_GLOBAL Ctrl* C = gconst(s.ctrl);
  if (C->status != ST_RUNNING) return;
  const int U0 = s.c0_U[0], U1 = s.c0_U[1], U2 = s.c0_U[2];
  const int64_t t = (int64_t)w.y * C0_TILE + threadIdx.x;
  if (t >= (int64_t)U0 * U1 * U2) return;
  const int k0 = (int)(t % U0);
  const int64_t r = t / U0;
  const int k1 = (int)(r % U1), k2 = (int)(r / U1);
  const int k[3] = {k0, k1, k2};
  double sv[3], cv[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    sv[a] = s.c0_sc[a][k[a]];
    cv[a] = s.c0_sc[a][s.c0_U[a] + k[a]];
  }
  const R f = (R)(2.0 / s.h);
  R re[3], im[3];
  re[0] = f * (R)(sv[0] * cv[1] * cv[2]);
  re[1] = f * (R)(cv[0] * sv[1] * cv[2]);
  re[2] = f * (R)(cv[0] * cv[1] * sv[2]);
  if (s.scheme == 1) {
    im[0] = f * (R)(cv[0] * sv[1] * sv[2]);
    im[1] = f * (R)(sv[0] * cv[1] * sv[2]);
    im[2] = f * (R)(sv[0] * sv[1] * cv[2]);
  } else {
    im[0] = im[1] = im[2] = 0;
  }
  const R xi2 = re[0] * re[0] + re[1] * re[1] + re[2] * re[2] + im[0] * im[0] + im[1] * im[1] + im[2] * im[2];
  // gather the components (absent coefficients are zero)
  int64_t off[3];
  bool has[3];
  cx<R> y[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    int l[3];
    bool ok = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      l[a] = k[a] - s.c0_off[q][a];
      ok = ok && l[a] >= 0 && l[a] < s.c0_M[q][a];
    }
    has[q] = ok;
    off[q] = ok ? ((int64_t)l[2] * s.c0_M[q][1] + l[1]) * s.c0_M[q][0] + l[0] : 0;
    cx<R> v = mk<R>(0, 0);
    if (ok) {
      const FM_GLOBAL R* b = gconst((const R*)s.c0_spec[q]);
      if (s.c0_cplx) v = mk<R>(b[2 * off[q]], b[2 * off[q] + 1]);
      else v.re = b[off[q]];
    }
    y[q] = phase_mul<R>(v, s.c0_phase[q], false);
  }
  cx<R> u[3] = {mk<R>(0, 0), mk<R>(0, 0), mk<R>(0, 0)};
  if (xi2 != (R)0) {
    // small strain (Appendix A): K = mu0 |xi|^2 + (mu0 + lambda0) Re(xi xi^H);
    // finite strain (Eq. FourierSGO): K = 2 mu0 |xi|^2 + lambda0 Re(xi xi^H)
    const R mu0 = (R)(s.fs ? 2.0 * s.mu0 : s.mu0), b = (R)(s.fs ? s.lam0 : s.mu0 + s.lam0);
    R K[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) K[i][j] = b * (re[i] * re[j] + im[i] * im[j]) + (i == j ? mu0 * xi2 : (R)0);
    // inverse of the symmetric 3 x 3 matrix by cofactors
    const R c00 = K[1][1] * K[2][2] - K[1][2] * K[1][2];
    const R c01 = K[0][2] * K[1][2] - K[0][1] * K[2][2];
    const R c02 = K[0][1] * K[1][2] - K[0][2] * K[1][1];
    const R c11 = K[0][0] * K[2][2] - K[0][2] * K[0][2];
    const R c12 = K[0][1] * K[0][2] - K[0][0] * K[1][2];
    const R c22 = K[0][0] * K[1][1] - K[0][1] * K[0][1];
    const R det = K[0][0] * c00 + K[0][1] * c01 + K[0][2] * c02;
    const R id = (R)1 / det;
    const R Ki[3][3] = {{c00 * id, c01 * id, c02 * id}, {c01 * id, c11 * id, c12 * id}, {c02 * id, c12 * id, c22 * id}};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      cx<R> a = mk<R>(0, 0);
#pragma unroll
      for (int i = 0; i < 3; ++i) a = add(a, scl(y[i], Ki[q][i]));
      u[q] = phase_mul<R>(a, s.c0_phase[q], true);
    }
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    if (!has[q]) continue;
    FM_GLOBAL R* b = gmut((R*)s.c0_spec[q]);
    if (s.c0_cplx) {
      b[2 * off[q]] = u[q].re;
      b[2 * off[q] + 1] = u[q].im;
    } else {
      b[off[q]] = u[q].re;
    }
  }
}

}  // namespace fm

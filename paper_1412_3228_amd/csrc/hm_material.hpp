// Filtered stiffness c~ at one voxel (Section 2: c~(x_a) = HR(c, omega(x_a))
// with the Voigt rule of eq. 3, the Reuss rule of eq. 4 and the 2-layer rule
// of eq. 5) and the polarization tau = (c~ - c0) : eps of eq. 1-b.
//
// Every c~ used here is written in one transversely isotropic form about a
// unit normal n (N = n (x) n):
//   sigma = a1 tr(eps) I + a2 eps + a3 [(n.eps.n) I + tr(eps) N]
//         + a4 (n.eps.n) N + a5 (N eps + eps N)
// Isotropic tensors (pure phases, Voigt, Reuss) have a3 = a4 = a5 = 0,
// a1 = lambda, a2 = 2 mu.  For the 2-layer rule of two isotropic layers
// with fractions g = 1 - f (matrix) and f (inclusion), <.> the
// fraction-weighted mean and M = lambda + 2 mu, the laminate stiffness in
// the normal frame is
//   C33 = 1/<1/M>, C13 = C33 <lambda/M>, C44 = 1/<1/mu>, C66 = <mu>,
//   C11 = <M - lambda^2/M> + C33 <lambda/M>^2,
//   C12 = <lambda - lambda^2/M> + C33 <lambda/M>^2,
// which is what the interface conditions of eq. 5-a (continuous
// out-of-plane stress, continuous in-plane strain) and the averages of
// eq. 5-b give; then a1 = C12, a2 = C11 - C12, a3 = C13 - C12,
// a4 = C33 + C11 - 2 C13 - 4 C44, a5 = 2 C44 - 2 C66.
#pragma once

#include "hm_common.hpp"

namespace hm {

enum : int { RULE_NONE = 0, RULE_VOIGT = 1, RULE_REUSS = 2, RULE_LAMINATE = 3 };

template <typename S> struct Coef {
  S a1, a2, a3, a4, a5;
  S n[3];
  bool aniso;
};

// Coefficients of the rule's formula at fraction f (no pure-phase shortcut),
// in scalar type S (a real or a dual number); pl/pm are the phase Lame
// parameters.  Isotropic rules leave n untouched.
template <typename S>
__device__ __forceinline__ void rule_coefficients(int rule, S f, const S pl[2], const S pm[2], Coef<S>& c) {
  const S g = S(1.0) - f;
  c.aniso = false;
  c.a3 = S(0.0);
  c.a4 = S(0.0);
  c.a5 = S(0.0);
  if (rule == RULE_REUSS) {
    const S K0 = pl[0] + S(2.0 / 3.0) * pm[0];
    const S K1 = pl[1] + S(2.0 / 3.0) * pm[1];
    const S K = S(1.0) / (g / K0 + f / K1);
    const S mu = S(1.0) / (g / pm[0] + f / pm[1]);
    c.a1 = K - S(2.0 / 3.0) * mu;
    c.a2 = S(2.0) * mu;
  } else if (rule == RULE_LAMINATE) {
    const S M0 = pl[0] + S(2.0) * pm[0];
    const S M1 = pl[1] + S(2.0) * pm[1];
    const S r0 = pl[0] / M0, r1 = pl[1] / M1;
    const S C33 = S(1.0) / (g / M0 + f / M1);
    const S lm = g * r0 + f * r1;
    const S C13 = C33 * lm;
    const S C44 = S(1.0) / (g / pm[0] + f / pm[1]);
    const S C66 = g * pm[0] + f * pm[1];
    const S q = C33 * lm * lm;
    const S C11 = g * (M0 - pl[0] * r0) + f * (M1 - pl[1] * r1) + q;
    const S C12 = g * (pl[0] - pl[0] * r0) + f * (pl[1] - pl[1] * r1) + q;
    c.a1 = C12;
    c.a2 = C11 - C12;
    c.a3 = C13 - C12;
    c.a4 = C33 + C11 - S(2.0) * C13 - S(4.0) * C44;
    c.a5 = S(2.0) * C44 - S(2.0) * C66;
    c.aniso = true;
  } else {  // Voigt (also used for fractional voxels under RULE_NONE)
    c.a1 = g * pl[0] + f * pl[1];
    c.a2 = S(2.0) * (g * pm[0] + f * pm[1]);
  }
}

// Unit normal from the centre of sphere k to the centre of voxel (x, y, z),
// voxel units, the difference folded once into [-n/2, n/2) per axis (Section
// 2 setup: normal linking the inclusion centre to x_a); e_1 when they coincide.
template <typename T>
__device__ __forceinline__ void interface_normal(const double* sph, int k, int x, int y, int z, int nx, int ny,
                                                 int nz, int dim, T n[3]) {
  double d[3];
  const double p[3] = {x + 0.5, y + 0.5, z + 0.5};
  const int nn[3] = {nx, ny, nz};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double v = p[a] - sph[4 * k + a];
    const double h = 0.5 * nn[a];
    if (v >= h) v -= nn[a];
    if (v < -h) v += nn[a];
    d[a] = v;
  }
  if (dim == 2) d[2] = 0.0;
  const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  if (r2 > 0.0) {
    const double inv = 1.0 / sqrt(r2);
    n[0] = T(d[0] * inv);
    n[1] = T(d[1] * inv);
    n[2] = T(d[2] * inv);
  } else {
    n[0] = T(1.0);
    n[1] = T(0.0);
    n[2] = T(0.0);
  }
}

// sigma = c : e for the transversely isotropic form above; e and s hold the
// tensor components (11, 22, 33, 23, 13, 12).
template <typename S>
__device__ __forceinline__ void apply_form(const Coef<S>& c, const S e[6], S s[6]) {
  const S tr = e[0] + e[1] + e[2];
  const S t = c.a1 * tr;
  s[0] = t + c.a2 * e[0];
  s[1] = t + c.a2 * e[1];
  s[2] = t + c.a2 * e[2];
  s[3] = c.a2 * e[3];
  s[4] = c.a2 * e[4];
  s[5] = c.a2 * e[5];
  if (c.aniso) {
    const S n0 = c.n[0], n1 = c.n[1], n2 = c.n[2];
    // (eps n)_i
    const S en0 = e[0] * n0 + e[5] * n1 + e[4] * n2;
    const S en1 = e[5] * n0 + e[1] * n1 + e[3] * n2;
    const S en2 = e[4] * n0 + e[3] * n1 + e[2] * n2;
    const S nen = en0 * n0 + en1 * n1 + en2 * n2;
    const S ai = c.a3 * nen;            // a3 (n.eps.n) I
    const S an = c.a3 * tr + c.a4 * nen;  // [a3 tr + a4 n.eps.n] N
    s[0] += ai + an * n0 * n0 + c.a5 * S(2.0) * n0 * en0;
    s[1] += ai + an * n1 * n1 + c.a5 * S(2.0) * n1 * en1;
    s[2] += ai + an * n2 * n2 + c.a5 * S(2.0) * n2 * en2;
    s[3] += an * n1 * n2 + c.a5 * (n1 * en2 + en1 * n2);
    s[4] += an * n0 * n2 + c.a5 * (n0 * en2 + en0 * n2);
    s[5] += an * n0 * n1 + c.a5 * (n0 * en1 + en0 * n1);
  }
}

}  // namespace hm

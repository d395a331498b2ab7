// gfx950 kernels of the mesh-transform renderer.
//
// Method (paper Sec. 4): the transform of a triangle T at frequency xi is
// 2 A_T f_T(xi) with f_T the second divided difference of exp at the nodes
// z_p = -i v_p.xi (Eq. 7-8); its vertex derivatives are third divided
// differences with a repeated node (Eq. 9-10).  Near-coincident phases
// (Sec. 4.1.3) are handled here by two evaluation schemes that are exact in
// real arithmetic and stable in float32:
//   * nodes spread by less than one radian: a series about the node mean,
//     written in the elementary symmetric polynomials E2, E3 of the centred
//     phases (complete homogeneous polynomials h_n of the nodes divided by
//     (n+2)!);
//   * otherwise: the nodes are sorted, DD3 = [DD2(mid,hi) - DD2(lo,mid)] /
//     (z_hi - z_lo) with each DD2 in its sinc form, and the repeated-node
//     DD4 from the same recurrence with the second phi-function
//     phi2(z) = (e^z - 1 - z)/z^2.
// Vertex phases are carried in revolutions (k . u with integer k and u =
// x / L), so the large part of every phase is reduced exactly before the
// hardware sine and cosine (v_sin_f32 / v_cos_f32 take revolutions); the
// closed forms take the phases of two vertices relative to the third in
// radians, small numbers computed from the edges.
//
// Work layout: both sweeps put band frequencies on lanes and stream triangle
// records as wave-uniform values.  The gradient
// sweep evaluates most pairs in the closed Lagrange form and queues the pairs
// with nearly coincident nodes in LDS for the stable scheme above, so the
// stable branch runs on full waves.  Every reduction is a fixed-order sum (no
// float atomics), so results are bitwise reproducible.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "dm_internal.h"

namespace dm {

namespace {

constexpr float TWO_PI_F = 6.283185307179586477f;
constexpr float PI_F = 3.141592653589793238f;
constexpr double TWO_PI_D = 6.283185307179586476925286766559;
// Series branch when the node spread is below one radian.
constexpr float SERIES_REV = 0.15915494309189535f;   // 1 / (2 pi)
constexpr float INV_TWO_PI_F = 0.15915494309189535f;
// Closed (Lagrange) form of the gradient pair when every node gap is at least
// 0.01 revolutions and the spread at least one radian; other pairs go to
// vjp_pair_series / vjp_pair_sorted.  Its float32 rounding grows like 1 / (2 pi gap)^2; at this gap the
// vertex gradients stay within about 1e-5 relative of the float64 result, an
// order of magnitude inside the gradient tolerance.  The main loops compare
// relative phases in radians.
constexpr float LAG_GAP_RAD = 0.06283185307179587f;   // 0.01 rev
constexpr float SERIES_RAD = 1.0f;
// Below one radian of spread the closed form is still used when the smallest
// gap times the spread is at least LAG_GAP_SPREAD: its float32 error grows like
// 1 / (smallest gap x spread), so those pairs are no less accurate than pairs
// at the gap threshold with a spread of one radian or more.
constexpr float LAG_GAP_SPREAD = LAG_GAP_RAD * SERIES_RAD;

// e^{-2 pi i r} for r in revolutions, r already in [-1/2, 1/2].
__device__ __forceinline__ void cis_neg(float r, float& c, float& s_neg) {
  c = __builtin_amdgcn_cosf(r);
  s_neg = -__builtin_amdgcn_sinf(r);
}

// Branch-free select: both operands are materialised before the choice, so
// the compiler emits v_cndmask instead of a divergent branch.
__device__ __forceinline__ float pick(bool c, float a, float b) {
  asm volatile("" : "+v"(a), "+v"(b));
  return c ? a : b;
}

// A polynomial coefficient of the stable schemes, made opaque where it is
// used.  Those schemes run only in the queue passes; with plain literals the
// compiler materialises their coefficients in vector registers once, ahead
// of the sweep loops, and keeps them live through the main loop, where the
// registers are needed.
__device__ __forceinline__ float kc(float c) {
  asm volatile("" : "+s"(c));
  return c;
}

// sin(x)/x for x >= 0 given sin(x): polynomial below 0.5, quotient above.
__device__ __forceinline__ float sinc_from(float x, float sinx, float inv_x) {
  const float x2 = x * x;
  const float p = fmaf(x2, fmaf(x2, fmaf(x2, kc(-1.9841269841e-4f), kc(8.3333333333e-3f)), kc(-0.16666666667f)), 1.0f);
  return pick(x < 0.5f, p, sinx * inv_x);
}

// Integer-frequency phase of the record's vertex 3 (revolutions, integer
// part removed exactly) and the phases of vertices 2 and 3 relative to 1.
__device__ __forceinline__ float vertex3_phase(float kx, float ky, float kz, const float* r) {
  float th = fmaf(kz, r[2], fmaf(ky, r[1], kx * r[0]));   // exact: 12-bit grid part
  th -= __builtin_rintf(th);
  return th + fmaf(kz, r[5], fmaf(ky, r[4], kx * r[3]));
}
// w - k.u3 up to an integer (revolutions): the fraction of the exact grid
// part (v_fract is exact there), then the rest, with w (a phase in
// revolutions, e.g. the adjoint weight's, at most 1/2 in magnitude) folded
// into it.  The rest is at most sum |k_j| / 8192 + 1/2 in magnitude, so with
// at most 2^20 samples per grid axis the result lies within (-194, 194): the
// hardware sine and cosine take it as it is (their domain is [-256, 256]
// revolutions, and on the device they agree with the argument wrapped into
// [0, 1), more closely near zero, where the wrap loses the low bits).
__device__ __forceinline__ float vertex3_wphase(float kx, float ky, float kz, const float* r, float w) {
  const float th = fmaf(kz, r[2], fmaf(ky, r[1], kx * r[0]));   // exact: 12-bit grid part
  const float lo = fmaf(kz, r[5], fmaf(ky, r[4], fmaf(kx, r[3], -w)));
  return __builtin_amdgcn_fractf(-th) - lo;
}
// Phases of vertices 2 and 3 relative to vertex 1 in radians (the record
// holds the edges times 2 pi / L).
__device__ __forceinline__ void rel_phases(float kx, float ky, float kz, const float* r, float& d2, float& d3) {
  d2 = fmaf(kz, r[8], fmaf(ky, r[7], kx * r[6]));
  d3 = fmaf(kz, r[11], fmaf(ky, r[10], kx * r[9]));
}
// The same in revolutions.
__device__ __forceinline__ void rel_phases_rev(float kx, float ky, float kz, const float* r, float& d2, float& d3) {
  rel_phases(kx, ky, kz, r, d2, d3);
  d2 *= INV_TWO_PI_F;
  d3 *= INV_TWO_PI_F;
}
// Phase of vertex 1 and the two relative phases (revolutions).
__device__ __forceinline__ void tri_phases(float kx, float ky, float kz, const float* r, float& t1, float& d2,
                                           float& d3) {
  rel_phases_rev(kx, ky, kz, r, d2, d3);
  t1 = vertex3_phase(kx, ky, kz, r) - d3;
}

// Wrap revolutions into [0, 1) for the hardware sine/cosine (v_fract_f32).
__device__ __forceinline__ float wrap(float r) { return __builtin_amdgcn_fractf(r); }

// Series coefficients of DD3 about the node mean (centred phases a_p,
// E2 = sum a_p a_q, E3 = a_0 a_1 a_2):  Phi = pre + i pim.
__device__ __forceinline__ void series_phi(float E2, float E3, float& pre, float& pim) {
  const float c6 = kc(2.4801587302e-5f);
  pre = fmaf(E2, fmaf(E2, fmaf(E2, c6, kc(1.3888888889e-3f)), kc(4.1666666667e-2f)), 0.5f) - E3 * E3 * c6;
  pim = E3 * fmaf(E2, fmaf(E2, kc(8.2671957672e-6f), kc(3.9682539683e-4f)), kc(8.3333333333e-3f));
}

// Reciprocals of S = 2 pi s and of the half gaps x1, x2 clamped at 1/2 (the
// quotients are only used where x >= 1/2), from one v_rcp_f32.
struct Recips {
  float invS, invX1, invX2;
};
__device__ __forceinline__ Recips recips(float S, float x1, float x2) {
  const float X1 = fmaxf(x1, 0.5f), X2 = fmaxf(x2, 0.5f);
  const float X12 = X1 * X2;
  const float rinv = __builtin_amdgcn_rcpf(S * X12);
  const float rS = rinv * S;
  return {rinv * X12, rS * X2, rS * X1};
}

// acc += w f_T, f_T = DD3[exp](-2 pi i (t1 + {0, d2, d3})).
//   dd3_acc_series, for a spread below 1 rad: series about the node mean;
//   dd3_acc_sorted, otherwise (sorted nodes):  f = (i/S) [sinc(pi g2) e^{-2 pi i m_mh} - sinc(pi g1) e^{-2 pi i m_lm}]
//   with m_lm, m_mh the phases at the midpoints of the lo-mid and mid-hi edges.
__device__ __forceinline__ void dd3_acc_series(float t1, float d2, float d3, float w, float& ar, float& ai) {
  const float m = (d2 + d3) * (1.0f / 3.0f);
  const float a0 = -TWO_PI_F * m, a1 = TWO_PI_F * (d2 - m), a2 = TWO_PI_F * (d3 - m);
  float pre, pim;
  series_phi(fmaf(a0, a1 + a2, a1 * a2), a0 * a1 * a2, pre, pim);
  const float r = wrap(t1 + m);
  const float c = __builtin_amdgcn_cosf(r), sn = -__builtin_amdgcn_sinf(r);
  ar = fmaf(w, c * pre - sn * pim, ar);
  ai = fmaf(w, fmaf(c, pim, sn * pre), ai);
}

__device__ __forceinline__ void dd3_acc_sorted(float t1, float d2, float d3, float w, float& ar, float& ai) {
  const float lo = fminf(fminf(0.0f, d2), d3);
  const float hi = fmaxf(fmaxf(0.0f, d2), d3);
  const float s = hi - lo;
  const float mid = __builtin_amdgcn_fmed3f(0.0f, d2, d3);
  const float g1 = mid - lo, g2 = hi - mid;
  const float x1 = PI_F * g1, x2 = PI_F * g2;
  const Recips q = recips(TWO_PI_F * s, x1, x2);
  const float sg1 = sinc_from(x1, __builtin_amdgcn_sinf(wrap(0.5f * g1)), q.invX1);
  const float sg2 = sinc_from(x2, __builtin_amdgcn_sinf(wrap(0.5f * g2)), q.invX2);
  const float rlm = wrap(fmaf(0.5f, lo + mid, t1)), rmh = wrap(fmaf(0.5f, mid + hi, t1));
  const float clm = __builtin_amdgcn_cosf(rlm), slm = __builtin_amdgcn_sinf(rlm);
  const float cmh = __builtin_amdgcn_cosf(rmh), smh = __builtin_amdgcn_sinf(rmh);
  // B = sg2 E_mh - sg1 E_lm with E = (cos, -sin);  f = (i/S) B = (-B_i, B_r)/S
  const float br = fmaf(sg2, cmh, -sg1 * clm);
  const float bi = fmaf(sg1, slm, -sg2 * smh);
  const float c = w * q.invS;
  ar = fmaf(-c, bi, ar);
  ai = fmaf(c, br, ai);
}

// Either scheme, chosen per pair by the spread.
__device__ __forceinline__ void dd3_acc(float t1, float d2, float d3, float w, float& ar, float& ai) {
  const float s = fmaxf(fmaxf(0.0f, d2), d3) - fminf(fminf(0.0f, d2), d3);
  if (s < SERIES_REV)
    dd3_acc_series(t1, d2, d3, w, ar, ai);
  else
    dd3_acc_sorted(t1, d2, d3, w, ar, ai);
}

// One pair of the gradient sweep: with W the adjoint weight of the frequency,
//   VOLUME:  z[p]  = Re(W DD4_p)            (p over the slots {node 0, d2, d3})
//   SURFACE: wf    = Re(W f_T), z[p] = Im(W DD4_p)
// and in both modes fr + i fi = f_T (the fused sweep's forward value).
// DD4_p is the divided difference with node p repeated (Eq. 10 up to -i xi).
// Stable branch (sorted nodes, R = i/S, P_x = e^{-2 pi i t_x} the vertex phases,
// phi1, phi2 the first two phi-functions at -i Gamma_j):
//   f      = R (P_mid phi1(G2) - P_lo phi1(G1))
//   DD4_lo = R (f - P_lo phi2(G1)),  DD4_hi = R (P_hi conj phi2(G2) - f),
//   DD4_mid = R P_mid (phi2(G2) - conj phi2(G1)).
// Spread below one radian: the series about the node mean (vjp_pair_series);
// otherwise the sorted scheme (vjp_pair_sorted).  The gradient sweep queues
// the two kinds of pairs apart, so each pass runs one scheme only.
template <int MODE>
__device__ __forceinline__ void vjp_pair_series(float t1, float d2, float d3, float wr, float wi, float& wf,
                                                float z[3], float& fr, float& fi) {
  {
    const float m = (d2 + d3) * (1.0f / 3.0f);
    const float a[3] = {-TWO_PI_F * m, TWO_PI_F * (d2 - m), TWO_PI_F * (d3 - m)};
    const float E2 = fmaf(a[0], a[1] + a[2], a[1] * a[2]);
    const float E3 = a[0] * a[1] * a[2];
    float pre, pim;
    series_phi(E2, E3, pre, pim);
    // d Phi / d e2 and d Phi / d e3 (e2 = -E2, e3 = i E3 of the centred nodes)
    const float p2r = fmaf(E2, fmaf(E2, kc(-7.4404761905e-5f), kc(-2.7777777778e-3f)), kc(-4.1666666667e-2f));
    const float p2i = -E3 * fmaf(E2, kc(1.6534391534e-5f), kc(3.9682539683e-4f));
    const float p3r = fmaf(E2, fmaf(E2, kc(8.2671957672e-6f), kc(3.9682539683e-4f)), kc(8.3333333333e-3f));
    const float p3i = E3 * fmaf(E2, kc(1.6534391534e-6f), kc(4.9603174603e-5f));
    const float r = wrap(t1 + m);
    const float c = __builtin_amdgcn_cosf(r), sn = -__builtin_amdgcn_sinf(r);
    // WG = W e^{-2 pi i (t1 + m)}
    const float gr = wr * c - wi * sn, gi = fmaf(wr, sn, wi * c);
    if (MODE == 1) wf = gr * pre - gi * pim;
    fr = c * pre - sn * pim;
    fi = fmaf(c, pim, sn * pre);
    const float third_re = pre * (1.0f / 3.0f), third_im = pim * (1.0f / 3.0f);
    const float e2_23 = E2 * (2.0f / 3.0f);
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      const float b = fmaf(a[p], a[p], e2_23);
      const float Ar = third_re - a[p] * p2i - b * p3r;
      const float Ai = fmaf(a[p], p2r, third_im) - b * p3i;
      z[p] = MODE == 0 ? gr * Ar - gi * Ai : fmaf(gr, Ai, gi * Ar);
    }
  }
}

template <int MODE>
__device__ __forceinline__ void vjp_pair_sorted(float t1, float d2, float d3, float wr, float wi, float& wf,
                                                float z[3], float& fr, float& fi) {
  const float lo = fminf(fminf(0.0f, d2), d3);
  const float hi = fmaxf(fmaxf(0.0f, d2), d3);
  const float s = hi - lo;
  const float mid = __builtin_amdgcn_fmed3f(0.0f, d2, d3);
  const float g1 = mid - lo, g2 = hi - mid;
  const float x1 = PI_F * g1, x2 = PI_F * g2;
  const Recips q = recips(TWO_PI_F * s, x1, x2);
  const float b1 = wrap(0.5f * g1), b2 = wrap(0.5f * g2), bl = wrap(t1 + lo);
  const float c1 = __builtin_amdgcn_cosf(b1), s1 = __builtin_amdgcn_sinf(b1);   // h1 = (c1, -s1)
  const float c2 = __builtin_amdgcn_cosf(b2), s2 = __builtin_amdgcn_sinf(b2);   // h2 = (c2, -s2)
  const float plr = __builtin_amdgcn_cosf(bl), pli = -__builtin_amdgcn_sinf(bl);  // P_lo
  const float sg1 = sinc_from(x1, s1, q.invX1), sg2 = sinc_from(x2, s2, q.invX2);
  // psi(G) = (G - sin G) / G^2: series below G = 1, quotient above (sin G = 2 s c)
  float psi1, psi2;
  {
    const float G = 2.0f * x1, G2 = G * G;
    const float ser = G * fmaf(G2, fmaf(G2, fmaf(G2, kc(-2.7557319224e-6f), kc(1.9841269841e-4f)),
                                         kc(-8.3333333333e-3f)),
                               kc(0.16666666667f));
    const float ig = 0.5f * q.invX1;
    psi1 = pick(x1 < 0.5f, ser, fmaf(-2.0f * s1, c1, G) * ig * ig);
  }
  {
    const float G = 2.0f * x2, G2 = G * G;
    const float ser = G * fmaf(G2, fmaf(G2, fmaf(G2, kc(-2.7557319224e-6f), kc(1.9841269841e-4f)),
                                         kc(-8.3333333333e-3f)),
                               kc(0.16666666667f));
    const float ig = 0.5f * q.invX2;
    psi2 = pick(x2 < 0.5f, ser, fmaf(-2.0f * s2, c2, G) * ig * ig);
  }
  // P_mid = P_lo h1^2, P_hi = P_mid h2^2
  const float e1r = fmaf(c1, c1, -s1 * s1), e1i = -2.0f * c1 * s1;
  const float e2r = fmaf(c2, c2, -s2 * s2), e2i = -2.0f * c2 * s2;
  const float pmr = plr * e1r - pli * e1i, pmi = fmaf(plr, e1i, pli * e1r);
  const float phr = pmr * e2r - pmi * e2i, phi = fmaf(pmr, e2i, pmi * e2r);
  // phi1 = h sinc ; phi2 = sinc^2/2 - i psi
  const float q1r = c1 * sg1, q1i = -s1 * sg1, q2r = c2 * sg2, q2i = -s2 * sg2;
  const float f1r = 0.5f * sg1 * sg1, f1i = -psi1, f2r = 0.5f * sg2 * sg2, f2i = -psi2;
  // F0 = P_mid phi1_2 - P_lo phi1_1 ; f = (i/S) F0
  const float F0r = (pmr * q2r - pmi * q2i) - (plr * q1r - pli * q1i);
  const float F0i = fmaf(pmr, q2i, pmi * q2r) - fmaf(plr, q1i, pli * q1r);
  fr = -F0i * q.invS;
  fi = F0r * q.invS;
  // W' = W (i/S)
  const float Wr = -wi * q.invS, Wi = wr * q.invS;
  if (MODE == 1) wf = wr * fr - wi * fi;
  // brackets
  const float blr = fr - (plr * f1r - pli * f1i), bli = fi - fmaf(plr, f1i, pli * f1r);
  const float bhr = fmaf(phr, f2r, phi * f2i) - fr, bhi = (phi * f2r - phr * f2i) - fi;
  const float dr = f2r - f1r, di = f2i + f1i;
  const float bmr = pmr * dr - pmi * di, bmi = fmaf(pmr, di, pmi * dr);
  float zl, zh, zm;
  if (MODE == 0) {
    zl = Wr * blr - Wi * bli;
    zh = Wr * bhr - Wi * bhi;
    zm = Wr * bmr - Wi * bmi;
  } else {
    zl = fmaf(Wr, bli, Wi * blr);
    zh = fmaf(Wr, bhi, Wi * bhr);
    zm = fmaf(Wr, bmi, Wi * bmr);
  }
  const float v[3] = {0.0f, d2, d3};
#pragma unroll
  for (int p = 0; p < 3; ++p) z[p] = v[p] == lo ? zl : (v[p] == hi ? zh : zm);
}

// ------------------------------------------------------------- the band
__device__ __forceinline__ int fft_freq(int i, int n) { return i < (n + 1) / 2 ? i : i - n; }

#pragma clang fp contract(off)
__device__ __noinline__ double band_q(const double* S, const GridC& g, double kx, double ky, double kz) {
  const double x = (TWO_PI_D * kx) / g.L[0];
  const double y = (TWO_PI_D * ky) / g.L[1];
  const double z = (TWO_PI_D * kz) / g.L[2];
  double q = (S[0] * x) * x;
  q = q + (S[1] * y) * y;
  q = q + (S[2] * z) * z;
  q = q + 2.0 * ((S[3] * x) * y);
  q = q + 2.0 * ((S[4] * x) * z);
  q = q + 2.0 * ((S[5] * y) * z);
  return q;
}
#pragma clang fp contract(on)

struct Sig6 {
  double s[6];
};

// Bricks of 4x4x4 positions of the half spectrum, brick-major order: the 64
// entries of a wave stay close in frequency space.
__device__ __forceinline__ bool slot_pos(const GridC& g, int64_t slot, int& ix, int& iy, int& iz) {
  const int64_t b = slot >> 6;
  const int w = (int)(slot & 63);
  const int nbz = (g.n2h + 3) >> 2, nby = (g.n1 + 3) >> 2;
  const int bz = (int)(b % nbz);
  const int64_t r = b / nbz;
  const int by = (int)(r % nby);
  const int bx = (int)(r / nby);
  ix = bx * 4 + (w >> 4);
  iy = by * 4 + ((w >> 2) & 3);
  iz = bz * 4 + (w & 3);
  return ix < g.n0 && iy < g.n1 && iz < g.n2h;
}

struct Aliases {
  int n;                 // 1 or 2
  int k[2][3];
};

__device__ __forceinline__ Aliases aliases_of(const GridC& g, int ix, int iy, int iz) {
  Aliases a;
  const int kx = fft_freq(ix, g.n0), ky = fft_freq(iy, g.n1);
  const bool nz_even = (g.n2 & 1) == 0;
  const int kz = (nz_even && iz == g.n2 / 2) ? -iz : iz;
  const bool nyx = (g.n0 & 1) == 0 && ix == g.n0 / 2;
  const bool nyy = (g.n1 & 1) == 0 && iy == g.n1 / 2;
  const bool nyz = nz_even && iz == g.n2 / 2;
  a.k[0][0] = kx;
  a.k[0][1] = ky;
  a.k[0][2] = kz;
  a.n = (nyx || nyy || nyz) ? 2 : 1;
  a.k[1][0] = nyx ? -kx : kx;
  a.k[1][1] = nyy ? -ky : ky;
  a.k[1][2] = nyz ? -kz : kz;
  return a;
}

__global__ void k_band_count(GridC g, Sig6 S, double qmax, int32_t* __restrict__ cnt, int64_t n_slots) {
  const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= n_slots) return;
  int ix, iy, iz;
  int c = 0;
  if (slot_pos(g, slot, ix, iy, iz)) {
    const Aliases a = aliases_of(g, ix, iy, iz);
    for (int j = 0; j < a.n; ++j)
      c += band_q(S.s, g, a.k[j][0], a.k[j][1], a.k[j][2]) < qmax ? 1 : 0;
  }
  cnt[slot] = c;
}

__global__ void k_band_fill(GridC g, Sig6 S, double qmax, const int32_t* __restrict__ cnt,
                            const int32_t* __restrict__ off, int64_t n_slots, BandDev b) {
  const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= n_slots) return;
  int ix, iy, iz;
  if (!slot_pos(g, slot, ix, iy, iz)) return;
  const int p = (ix * g.n1 + iy) * g.n2h + iz;
  const int c = cnt[slot];
  if (c == 0) {
    b.map[p] = -1;
    return;
  }
  const int e0 = off[slot];
  b.map[p] = e0 | ((c - 1) << 30);
  const Aliases a = aliases_of(g, ix, iy, iz);
  int e = e0;
  for (int j = 0; j < a.n; ++j) {
    const double q = band_q(S.s, g, a.k[j][0], a.k[j][1], a.k[j][2]);
    if (!(q < qmax)) continue;
    b.kf[e] = make_float4((float)a.k[j][0], (float)a.k[j][1], (float)a.k[j][2], (float)exp(-0.5 * q));
    b.wgt[e] = a.n == 2 ? 0.5f : 1.0f;
    b.pos[e] = p;
    ++e;
  }
}

// Band of a tabulated OTF (a PSF given as an array of its transform): the
// half-spectrum positions whose value has Re^2 + Im^2 > tau^2, decided in
// float64 without contraction so that membership is reproducible.
#pragma clang fp contract(off)
__device__ __noinline__ bool otf_in_band(float2 o, double tau2) {
  const double re = o.x, im = o.y;
  return re * re + im * im > tau2;
}
#pragma clang fp contract(on)

__global__ void k_band_count_otf(GridC g, const float2* __restrict__ otf, double tau2, int32_t* __restrict__ cnt,
                                 int64_t n_slots) {
  const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= n_slots) return;
  int ix, iy, iz;
  int c = 0;
  if (slot_pos(g, slot, ix, iy, iz)) {
    const int p = (ix * g.n1 + iy) * g.n2h + iz;
    if (otf_in_band(otf[p], tau2)) c = aliases_of(g, ix, iy, iz).n;
  }
  cnt[slot] = c;
}

__global__ void k_band_fill_otf(GridC g, const float2* __restrict__ otf, double tau2,
                                const int32_t* __restrict__ cnt, const int32_t* __restrict__ off, int64_t n_slots,
                                BandDev b) {
  const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= n_slots) return;
  int ix, iy, iz;
  if (!slot_pos(g, slot, ix, iy, iz)) return;
  const int p = (ix * g.n1 + iy) * g.n2h + iz;
  const int c = cnt[slot];
  if (c == 0) {
    b.map[p] = -1;
    return;
  }
  const int e0 = off[slot];
  // the band's arrays hold b.n_entries entries (the count the caller planned
  // with); a table changed since that count must not write past them
  if ((int64_t)e0 + c > b.n_entries) {
    b.map[p] = -1;
    return;
  }
  b.map[p] = e0 | ((c - 1) << 30);
  const Aliases a = aliases_of(g, ix, iy, iz);
  for (int j = 0; j < a.n; ++j) {
    b.kf[e0 + j] = make_float4((float)a.k[j][0], (float)a.k[j][1], (float)a.k[j][2], 1.0f);
    b.wgt[e0 + j] = a.n == 2 ? 0.5f : 1.0f;
    b.pos[e0 + j] = p;
  }
}

// ------------------------------------------------------------- scan (int32)
constexpr int SCAN_T = 256, SCAN_PER = 4, SCAN_BLK = SCAN_T * SCAN_PER;

__device__ int block_excl_scan(int v, int* sh, int& total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int o = 1; o < SCAN_T; o <<= 1) {
    const int add = t >= o ? sh[t - o] : 0;
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  total = sh[SCAN_T - 1];
  const int incl = sh[t];
  __syncthreads();
  return incl - v;
}

__global__ void __launch_bounds__(SCAN_T) k_scan_reduce(const int32_t* __restrict__ in, int64_t n,
                                                          int32_t* __restrict__ bsum) {
  __shared__ int sh[SCAN_T];
  const int64_t base = (int64_t)blockIdx.x * SCAN_BLK + threadIdx.x * SCAN_PER;
  int v = 0;
  for (int j = 0; j < SCAN_PER; ++j)
    if (base + j < n) v += in[base + j];
  int total;
  block_excl_scan(v, sh, total);
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

__global__ void __launch_bounds__(SCAN_T) k_scan_top(int32_t* __restrict__ bsum, int64_t nb,
                                                       int64_t* __restrict__ total_out) {
  __shared__ int sh[SCAN_T];
  const int64_t per = (nb + SCAN_T - 1) / SCAN_T;
  const int64_t b0 = threadIdx.x * per;
  int v = 0;
  for (int64_t j = 0; j < per; ++j)
    if (b0 + j < nb) v += bsum[b0 + j];
  int total;
  int run = block_excl_scan(v, sh, total);
  for (int64_t j = 0; j < per; ++j)
    if (b0 + j < nb) {
      const int x = bsum[b0 + j];
      bsum[b0 + j] = run;
      run += x;
    }
  if (threadIdx.x == 0) *total_out = total;
}

__global__ void __launch_bounds__(SCAN_T) k_scan_apply(const int32_t* __restrict__ in, int32_t* __restrict__ out,
                                                         int64_t n, const int32_t* __restrict__ bsum) {
  __shared__ int sh[SCAN_T];
  const int64_t base = (int64_t)blockIdx.x * SCAN_BLK + threadIdx.x * SCAN_PER;
  int v[SCAN_PER];
  int s = 0;
  for (int j = 0; j < SCAN_PER; ++j) {
    v[j] = base + j < n ? in[base + j] : 0;
    s += v[j];
  }
  int total;
  int run = block_excl_scan(s, sh, total) + bsum[blockIdx.x];
  for (int j = 0; j < SCAN_PER; ++j) {
    if (base + j < n) out[base + j] = run;
    run += v[j];
  }
}

// --------------------------------------------------------------- mesh prep
constexpr int PREP_T = 256;

template <typename T>
__device__ T block_sum(T v, T* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int o = PREP_T / 2; o > 0; o >>= 1) {
    if (t < o) sh[t] += sh[t + o];
    __syncthreads();
  }
  const T r = sh[0];
  __syncthreads();
  return r;
}

__global__ void __launch_bounds__(PREP_T) k_prep_centroid(GridC g, const float* __restrict__ V, int nv,
                                                            MeshInfo* __restrict__ info) {
  __shared__ double sh[PREP_T];
  double a[3] = {0, 0, 0};
  for (int i = threadIdx.x; i < nv; i += PREP_T)
    for (int j = 0; j < 3; ++j) a[j] += (double)V[3 * i + j];
  double c[3];
  for (int j = 0; j < 3; ++j) c[j] = block_sum(a[j], sh) / (double)(nv > 0 ? nv : 1);
  if (threadIdx.x == 0) {
    for (int j = 0; j < 3; ++j) {
      info->c[j] = (float)c[j];
      info->cu[j] = ((double)(float)c[j] - g.origin[j]) / g.L[j];
    }
    info->pad0 = 0.0f;
  }
}

template <int MODE>
__global__ void __launch_bounds__(PREP_T) k_prep_tris(GridC g, const float* __restrict__ V,
                                                        const int32_t* __restrict__ F,
                                                        const int32_t* __restrict__ flags,
                                                        const float* __restrict__ tri_w, int nt,
                                                        const MeshInfo* __restrict__ info,
                                                        float* __restrict__ rec, double* __restrict__ tmp) {
  __shared__ double sh[PREP_T];
  double area = 0.0, vol = 0.0;
  const double c[3] = {(double)info->c[0], (double)info->c[1], (double)info->c[2]};
  for (int t = blockIdx.x * PREP_T + threadIdx.x; t < nt; t += gridDim.x * PREP_T) {
    double v[3][3];
    for (int p = 0; p < 3; ++p) {
      const int vi = F[3 * t + p];
      for (int j = 0; j < 3; ++j) v[p][j] = (double)V[3 * vi + j];
    }
    float* r = rec + (size_t)t * TRI_REC;
    double e2[3], e3[3], a[3], b[3];
    const int fl = flags[t];
    const double sgn = (fl & TRI_REVERSED) ? -1.0 : 1.0;
    // density weight (several materials or double membranes); 1 without weights
    const double wt = tri_w != nullptr ? (double)tri_w[t] : 1.0;
    for (int j = 0; j < 3; ++j) {
      const double u = (v[2][j] - c[j]) / g.L[j];
      const double uh = rint(u * (double)PHASE_GRID) / (double)PHASE_GRID;
      r[j] = (float)uh;
      r[3 + j] = (float)(u - uh);
      e2[j] = v[1][j] - v[0][j];
      e3[j] = v[2][j] - v[0][j];
      r[6 + j] = (float)(TWO_PI_D * e2[j] / g.L[j]);
      r[9 + j] = (float)(TWO_PI_D * e3[j] / g.L[j]);
      a[j] = v[1][j] - c[j];
      b[j] = v[2][j] - c[j];
    }
    const double n[3] = {sgn * (e2[1] * e3[2] - e2[2] * e3[1]), sgn * (e2[2] * e3[0] - e2[0] * e3[2]),
                         sgn * (e2[0] * e3[1] - e2[1] * e3[0])};
    const double twoA = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    if (MODE == 0) {
      for (int j = 0; j < 3; ++j) r[12 + j] = (float)(wt * n[j] / g.L[j]);
    } else {
      r[12] = (float)(wt * twoA);
      r[13] = 0.0f;
      r[14] = 0.0f;
    }
    r[15] = (fl & TRI_STRIP_START) ? 1.0f : 0.0f;
    area += wt * 0.5 * twoA;
    const double a0[3] = {v[0][0] - c[0], v[0][1] - c[1], v[0][2] - c[2]};
    vol += wt * sgn * (a0[0] * (a[1] * b[2] - a[2] * b[1]) + a0[1] * (a[2] * b[0] - a[0] * b[2]) +
                       a0[2] * (a[0] * b[1] - a[1] * b[0])) / 6.0;
  }
  area = block_sum(area, sh);
  vol = block_sum(vol, sh);
  if (threadIdx.x == 0) {
    tmp[2 * blockIdx.x] = area;
    tmp[2 * blockIdx.x + 1] = vol;
  }
}

__global__ void __launch_bounds__(PREP_T) k_prep_totals(const double* __restrict__ tmp, int nblk,
                                                          MeshInfo* __restrict__ info) {
  __shared__ double sh[PREP_T];
  double a = 0.0, v = 0.0;
  for (int i = threadIdx.x; i < nblk; i += PREP_T) {
    a += tmp[2 * i];
    v += tmp[2 * i + 1];
  }
  a = block_sum(a, sh);
  v = block_sum(v, sh);
  if (threadIdx.x == 0) {
    info->area = a;
    info->volume = v;
  }
}

// ------------------------------------------------------------ forward sweep
constexpr int SWEEP_T = 256;

// Forward sweep with band entries on lanes (FWD_J entries per lane; a block
// covers FWD_CHUNK entries) over a range of
// strip-ordered triangles.  Each triangle adds one vertex: its phase factor
// is computed, the other two are carried over from the previous triangle of
// the strip.  Pairs are evaluated in closed (Lagrange) form,
//   f = (-(b-a) E1 + b E2 - a E3) / (a b (b-a)),
// E_p = e^{-2 pi i t_p} (t_p in revolutions), a and b the phases of vertices
// 2 and 3 relative to vertex 1 in radians.  Pairs with a node gap below
// FWD_LAG_GAP_RAD or a spread below one radian are queued in LDS and
// evaluated by dd3_acc on full
// waves after every FWD_TQ triangles; their sums collect in an LDS row per
// entry and are added to the register sums at the end.
constexpr float FWD_LAG_GAP_RAD = 0.031415926535897934f;   // 0.005 rev
constexpr int FWD_TQ = 4;   // triangles whose queued pairs share one pass

// Queued pairs of FWD_TQ consecutive triangles share one pass.  Within a pass
// the sums are added to the per-entry LDS row triangle by triangle (a
// triangle queues each entry at most once), so no two lanes add to the same
// slot at once and the order of the additions is fixed.  Volume mode keeps two
// queues per wave, 0 for the series (spread below one radian) and 1 for the
// sorted scheme, flushed in that order, so a pass runs one scheme only; in
// surface mode queue 0 takes every pair and each lane picks its scheme (one
// queue measured faster there).
struct FwdLds {
  uint16_t queue[4][2][FWD_TQ * 64 * FWD_J];
  float2 fb[4][FWD_J][64];
};

// Forward-sweep queue item: triangle tag, entry step j and lane.  The lane is
// made opaque so that the item is built where it is stored, in the rarely
// taken append branches; otherwise the compiler keeps one precomputed item per
// step in a vector register through the whole main loop.
__device__ __forceinline__ uint16_t fwd_queue_item(int tag, int j, int lane) {
  asm volatile("" : "+v"(lane));
  return (uint16_t)((tag << 9) | (j << 6) | lane);
}
// Gradient-sweep queue item, the same fields.  The step is added by an
// opaque instruction, so that the item is built where it is stored, in the
// append branches; otherwise the compiler keeps one precomputed item per
// step in a vector register through the whole main loop.
__device__ __forceinline__ uint16_t queue_item(int tag, int j, int lane) {
  const int x = (tag << 9) | lane;
  if (j == 0) return (uint16_t)x;
  int y;
  asm volatile("v_or_b32 %0, %1, %2" : "=v"(y) : "n"(j << 6), "v"(x));
  return (uint16_t)y;
}
// The same item with the lane left visible to the compiler: the batched
// surface-density sweeps (gradient and fused) spill inside their triangle
// loops with the opaque form (the fused one 34 registers, 22 reloads per
// triangle, a third slower) and much less with this one, so those kernels use
// it.
__device__ __forceinline__ uint16_t plain_item(int tag, int j, int lane) {
  return (uint16_t)((tag << 9) | (j << 6) | lane);
}

// One triangle: X holds the phase factors of vertex 1, Y of vertex 2 (both
// computed here at a strip start); on return X holds those of vertex 3, so
// the next triangle of the strip is processed with the roles of X and Y
// swapped.  Pairs that need the stable scheme are appended to the queue with
// the triangle's tag (its offset in the group sharing a pass).
template <int MODE>
__device__ __forceinline__ void fwd_lanes_tri(const float* r, bool start, int tag, const float (&kx)[FWD_J],
                                              const float (&ky)[FWD_J], const float (&kz)[FWD_J], int rem,
                                              float (&Xr)[FWD_J], float (&Xi)[FWD_J], float (&Yr)[FWD_J],
                                              float (&Yi)[FWD_J], float (&ar)[FWD_J], float (&ai)[FWD_J], int lane,
                                              uint16_t (*queue)[FWD_TQ * 64 * FWD_J], int (&nq)[2]) {
  if (start) {
#pragma unroll
    for (int j = 0; j < FWD_J; ++j) {
      float d2, d3;
      rel_phases_rev(kx[j], ky[j], kz[j], r, d2, d3);
      const float t1 = vertex3_phase(kx[j], ky[j], kz[j], r) - d3;
      const float q1 = wrap(-t1), q2 = wrap(-(t1 + d2));
      Xr[j] = __builtin_amdgcn_cosf(q1);
      Xi[j] = __builtin_amdgcn_sinf(q1);
      Yr[j] = __builtin_amdgcn_cosf(q2);
      Yi[j] = __builtin_amdgcn_sinf(q2);
    }
  }
#pragma unroll
  for (int j = 0; j < FWD_J; ++j) {
    float a, b;
    rel_phases(kx[j], ky[j], kz[j], r, a, b);
    // e^{-2 pi i t} = (cos 2 pi q, sin 2 pi q) at q = -t: no negation of the sine
    const float q3 = vertex3_wphase(kx[j], ky[j], kz[j], r, 0.0f);
    const float Nr = __builtin_amdgcn_cosf(q3), Ni = __builtin_amdgcn_sinf(q3);
    const float c = b - a;
    const float mn = fminf(fminf(fabsf(a), fabsf(b)), fabsf(c));
    const float mx = fmaxf(fmaxf(fabsf(a), fabsf(b)), fabsf(c));
    const bool close = mn < FWD_LAG_GAP_RAD, small = mx < SERIES_RAD;
    const bool fast = !close && !small;
    // with the relative phases in radians the Lagrange quotient is f_T itself
    const float wt = MODE == 0 ? fmaf(kz[j], r[14], fmaf(ky[j], r[13], kx[j] * r[12])) : r[12];
    const float kk = fast ? wt * __builtin_amdgcn_rcpf(a * b * c) : 0.0f;
    const float tr = fmaf(-c, Xr[j], fmaf(b, Yr[j], -a * Nr));
    const float ti = fmaf(-c, Xi[j], fmaf(b, Yi[j], -a * Ni));
    ar[j] = fmaf(kk, tr, ar[j]);
    ai[j] = fmaf(kk, ti, ai[j]);
    // the lanes holding entries are the first cnt of the wave (cnt wave-uniform)
    const int cnt = rem - 64 * j;
    const bool valid = lane < cnt;
    const uint64_t vmask = cnt >= 64 ? ~0ull : (cnt <= 0 ? 0ull : (1ull << cnt) - 1ull);
    const uint64_t bs = __builtin_amdgcn_ballot_w64(MODE == 0 ? small : !fast) & vmask;
    const uint64_t bc = MODE == 0 ? __builtin_amdgcn_ballot_w64(close) & vmask & ~bs : 0ull;
    if (bs) {
      if ((MODE == 0 ? small : !fast) && valid) {
        const int pos = nq[0] + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bs >> 32),
                                                               __builtin_amdgcn_mbcnt_lo((uint32_t)bs, 0u));
        queue[0][pos] = fwd_queue_item(tag, j, lane);
      }
      nq[0] += __popcll(bs);
    }
    if (MODE == 0 && bc) {
      if (close && !small && valid) {
        const int pos = nq[1] + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bc >> 32),
                                                               __builtin_amdgcn_mbcnt_lo((uint32_t)bc, 0u));
        queue[1][pos] = fwd_queue_item(tag, j, lane);
      }
      nq[1] += __popcll(bc);
    }
    Xr[j] = Nr;
    Xi[j] = Ni;
  }
}

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Stable scheme (KIND 0 series, 1 sorted, 2 either) for the pairs of queue
// Q of the triangles starting at r (tag p = triangle r + p TRI_REC).
template <int MODE, int Q, int KIND>
__device__ __forceinline__ void fwd_lanes_flush(const float* r, const float4* __restrict__ kf, int64_t ew, int lane,
                                                int w, int nq, FwdLds& L) {
  wave_lds_sync();
  for (int q0 = 0; q0 < nq; q0 += 64) {
    const bool act = q0 + lane < nq;
    int p = -1, jj = 0, ll = 0;
    float fr = 0.0f, fi = 0.0f;
    if (act) {
      const int it = L.queue[w][Q][q0 + lane];
      p = it >> 9;
      jj = (it >> 6) & 7;
      ll = it & 63;
      const float* rp = r + (size_t)p * TRI_REC;
      const float4 k = kf[ew + 64 * jj + ll];
      float t1, d2, d3;
      tri_phases(k.x, k.y, k.z, rp, t1, d2, d3);
      const float wt = MODE == 0 ? fmaf(k.z, rp[14], fmaf(k.y, rp[13], k.x * rp[12])) : rp[12];
      if (KIND == 0)
        dd3_acc_series(t1, d2, d3, wt, fr, fi);
      else if (KIND == 1)
        dd3_acc_sorted(t1, d2, d3, wt, fr, fi);
      else
        dd3_acc(t1, d2, d3, wt, fr, fi);
    }
#pragma unroll
    for (int q = 0; q < FWD_TQ; ++q) {
      if (p == q) {
        float2& slot = L.fb[w][jj][ll];
        slot = make_float2(slot.x + fr, slot.y + fi);
      }
      wave_lds_sync();
    }
  }
}

template <int MODE>
__device__ __forceinline__ void fwd_lanes_tile(const float4* __restrict__ kf, int64_t nE, const float* __restrict__ rec,
                                               int t0, int t1, int64_t e_chunk, float2* __restrict__ part_row,
                                               FwdLds& L) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t ew = e_chunk + (int64_t)w * 64 * FWD_J;
  float kx[FWD_J], ky[FWD_J], kz[FWD_J], ar[FWD_J], ai[FWD_J];
  float Xr[FWD_J], Xi[FWD_J], Yr[FWD_J], Yi[FWD_J];
  // entries held by this wave: the first rem of its 64 FWD_J (wave-uniform)
  const int rem = __builtin_amdgcn_readfirstlane((int)max<int64_t>(0, min<int64_t>(nE - ew, 64 * FWD_J)));
#pragma unroll
  for (int j = 0; j < FWD_J; ++j) {
    const int64_t e = ew + 64 * j + lane;
    kx[j] = ky[j] = kz[j] = ar[j] = ai[j] = 0.0f;
    Xr[j] = Xi[j] = Yr[j] = Yi[j] = 0.0f;
    if (e < nE) {
      const float4 k = kf[e];
      kx[j] = k.x;
      ky[j] = k.y;
      kz[j] = k.z;
    }
    L.fb[w][j][lane] = make_float2(0.0f, 0.0f);
  }
  for (int t = t0; t < t1; t += FWD_TQ) {
    const float* r = rec + (size_t)t * TRI_REC;
    int nq[2] = {0, 0};
    // triangles t, t+1, ... alternate the roles of X and Y (see fwd_lanes_tri)
    fwd_lanes_tri<MODE>(r, t == t0 || r[15] != 0.0f, 0, kx, ky, kz, rem, Xr, Xi, Yr, Yi, ar, ai, lane, L.queue[w], nq);
    if (t + 1 < t1)
      fwd_lanes_tri<MODE>(r + TRI_REC, r[TRI_REC + 15] != 0.0f, 1, kx, ky, kz, rem, Yr, Yi, Xr, Xi, ar, ai, lane,
                          L.queue[w], nq);
    if (t + 2 < t1)
      fwd_lanes_tri<MODE>(r + 2 * TRI_REC, r[2 * TRI_REC + 15] != 0.0f, 2, kx, ky, kz, rem, Xr, Xi, Yr, Yi, ar, ai,
                          lane, L.queue[w], nq);
    if (t + 3 < t1)
      fwd_lanes_tri<MODE>(r + 3 * TRI_REC, r[3 * TRI_REC + 15] != 0.0f, 3, kx, ky, kz, rem, Yr, Yi, Xr, Xi, ar, ai,
                          lane, L.queue[w], nq);
    if (MODE == 0) {
      fwd_lanes_flush<MODE, 0, 0>(r, kf, ew, lane, w, nq[0], L);
      fwd_lanes_flush<MODE, 1, 1>(r, kf, ew, lane, w, nq[1], L);
    } else {
      fwd_lanes_flush<MODE, 0, 2>(r, kf, ew, lane, w, nq[0], L);
    }
  }
#pragma unroll
  for (int j = 0; j < FWD_J; ++j) {
    const int64_t e = ew + 64 * j + lane;
    if (e < nE) {
      const float2 f = L.fb[w][j][lane];
      part_row[e] = make_float2(ar[j] + f.x, ai[j] + f.y);
    }
  }
}

template <int MODE>
__global__ void __launch_bounds__(SWEEP_T, 7) k_fwd_lanes(const float4* __restrict__ kf, int64_t nE,
                                                         const float* __restrict__ rec, int nt, int tpc,
                                                         float2* __restrict__ part) {
  __shared__ FwdLds L;
  const int t0 = blockIdx.y * tpc;
  fwd_lanes_tile<MODE>(kf, nE, rec, t0, min(nt, t0 + tpc), (int64_t)blockIdx.x * FWD_CHUNK,
                       part + (size_t)blockIdx.y * nE, L);
}

// Phase factor e^{-i xi.(c - origin)} for integer frequency k (float32 after
// an exact float64 reduction).
__device__ __forceinline__ void ref_phase(const MeshInfo* info, float kx, float ky, float kz, float& pr,
                                          float& pi) {
  double t = (double)kx * info->cu[0] + (double)ky * info->cu[1] + (double)kz * info->cu[2];
  t -= rint(t);
  cis_neg((float)t, pr, pi);
}

// u_hat at one band entry from the summed sweep value.
template <int MODE>
__device__ __forceinline__ float2 finish_u(const GridC& g, const MeshInfo* info, float kx, float ky, float kz,
                                           float sr, float si) {
  float pr, pi;
  ref_phase(info, kx, ky, kz, pr, pi);
  const float zr = pr * sr - pi * si, zi = fmaf(pr, si, pi * sr);
  if (MODE == 0) {
    if (kx == 0.0f && ky == 0.0f && kz == 0.0f) return make_float2((float)info->volume, 0.0f);
    const float xx = kx * g.two_pi_over_L[0], xy = ky * g.two_pi_over_L[1], xz = kz * g.two_pi_over_L[2];
    const float q2 = fmaf(xz, xz, fmaf(xy, xy, xx * xx));
    const float f = TWO_PI_F / q2;   // u = i (2 pi / |xi|^2) z
    return make_float2(-zi * f, zr * f);
  }
  const float ia = (float)(1.0 / info->area);
  return make_float2(zr * ia, zi * ia);
}

template <int MODE>
__global__ void k_fwd_finalize(GridC g, BandDev b, const float2* __restrict__ part, int n_chunks,
                               const MeshInfo* __restrict__ info, float2* __restrict__ spec_out,
                               float2* __restrict__ xhalf) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= b.n_pos) return;
  const int32_t m = b.map[p];
  float xr = 0.0f, xi = 0.0f;
  if (m >= 0) {
    const int e0 = m & 0x3fffffff, cntm1 = (m >> 30) & 1;
    for (int e = e0; e <= e0 + cntm1; ++e) {
      float sr = 0.0f, si = 0.0f;
      for (int c = 0; c < n_chunks; ++c) {
        const float2 v = part[(size_t)c * b.n_entries + e];
        sr += v.x;
        si += v.y;
      }
      const float4 k = b.kf[e];
      const float2 u = finish_u<MODE>(g, info, k.x, k.y, k.z, sr, si);
      if (spec_out) spec_out[e] = u;
      const float hw = b.otf ? b.wgt[e] : k.w * b.wgt[e];
      xr = fmaf(hw, u.x, xr);
      xi = fmaf(hw, u.y, xi);
    }
    if (b.otf) {   // one tabulated value per position, shared by its aliases
      const float2 o = b.otf[p];
      const float tr = xr * o.x - xi * o.y;
      xi = fmaf(xr, o.y, xi * o.x);
      xr = tr;
    }
  }
  if (xhalf) xhalf[p] = make_float2(xr * g.inv_LV, xi * g.inv_LV);
}

__global__ void k_spec_scatter(GridC g, BandDev b, const float2* __restrict__ spec, float2* __restrict__ xhalf) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= b.n_pos) return;
  const int32_t m = b.map[p];
  float xr = 0.0f, xi = 0.0f;
  if (m >= 0) {
    const int e0 = m & 0x3fffffff, cntm1 = (m >> 30) & 1;
    for (int e = e0; e <= e0 + cntm1; ++e) {
      const float hw = b.otf ? b.wgt[e] : b.kf[e].w * b.wgt[e];
      xr = fmaf(hw, spec[e].x, xr);
      xi = fmaf(hw, spec[e].y, xi);
    }
    if (b.otf) {
      const float2 o = b.otf[p];
      const float tr = xr * o.x - xi * o.y;
      xi = fmaf(xr, o.y, xi * o.x);
      xr = tr;
    }
  }
  xhalf[p] = make_float2(xr * g.inv_LV, xi * g.inv_LV);
}

// ------------------------------------------------------- adjoint weights
constexpr int ADJ_T = 256;

template <int MODE>
__global__ void k_adjoint(GridC g, BandDev b, const float2* __restrict__ ghat, const MeshInfo* __restrict__ info,
                          float4* __restrict__ erec) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= b.n_pos) return;
  const int32_t m = b.map[p];
  if (m < 0) return;
  const float inv_area = MODE == 1 ? (float)(1.0 / info->area) : 1.0f;
  const int iz = (int)(p % g.n2h);
  const float cp = (iz == 0 || ((g.n2 & 1) == 0 && iz == g.n2 / 2)) ? 1.0f : 2.0f;
  const float2 G = ghat[p];
  const int e0 = m & 0x3fffffff, cntm1 = (m >> 30) & 1;
  for (int e = e0; e <= e0 + cntm1; ++e) {
    const float4 k = b.kf[e];
    float pr, pi;
    ref_phase(info, k.x, k.y, k.z, pr, pi);
    // W = c_p w_alias h_hat conj(G) e^{-i xi.(c-o)} / (Lx Ly Lz) [/ area]
    // (a tabulated OTF value multiplies as a complex number)
    const float a = cp * b.wgt[e] * (b.otf ? 1.0f : k.w) * g.inv_LV * inv_area;
    float wr = a * (G.x * pr + G.y * pi);
    float wi = a * (G.x * pi - G.y * pr);
    if (b.otf) {
      const float2 o = b.otf[p];
      const float tr = wr * o.x - wi * o.y;
      wi = fmaf(wr, o.y, wi * o.x);
      wr = tr;
    }
    erec[ERC * e] = make_float4(k.x, k.y, k.z, wr);
    erec[ERC * e + 1] = make_float4(wi, k.x * g.two_pi_over_L[0], k.y * g.two_pi_over_L[1], k.z * g.two_pi_over_L[2]);
    erec[ERC * e + 2] = make_float4(sqrtf(fmaf(wr, wr, wi * wi)), atan2f(wi, wr) * INV_TWO_PI_F, 0.0f, 0.0f);
  }
}

// PSF gradient partials: dL/dSigma_ab = sum_k c_p w h_hat Re[conj(G) u] (-1/2 xi_a xi_b)(2 - delta_ab) / LV,
// block sums in float64, reduced in a fixed order by k_dsig_final.
__global__ void __launch_bounds__(ADJ_T) k_dsig(GridC g, BandDev b, const float2* __restrict__ ghat,
                                                  const float2* __restrict__ spec, double* __restrict__ dsig_part) {
  __shared__ double sh[ADJ_T];
  double d6[6] = {0, 0, 0, 0, 0, 0};
  for (int64_t p = (int64_t)blockIdx.x * ADJ_T + threadIdx.x; p < b.n_pos; p += (int64_t)gridDim.x * ADJ_T) {
    const int32_t m = b.map[p];
    if (m < 0) continue;
    const int iz = (int)(p % g.n2h);
    const float cp = (iz == 0 || ((g.n2 & 1) == 0 && iz == g.n2 / 2)) ? 1.0f : 2.0f;
    const float2 G = ghat[p];
    const int e0 = m & 0x3fffffff, cntm1 = (m >> 30) & 1;
    for (int e = e0; e <= e0 + cntm1; ++e) {
      const float4 k = b.kf[e];
      const float2 u = spec[e];
      const double val = (double)(cp * b.wgt[e] * k.w * g.inv_LV) * (double)(G.x * u.x + G.y * u.y);
      const double X = k.x * g.two_pi_over_L[0], Y = k.y * g.two_pi_over_L[1], Z = k.z * g.two_pi_over_L[2];
      d6[0] += val * (-0.5 * X * X);
      d6[1] += val * (-0.5 * Y * Y);
      d6[2] += val * (-0.5 * Z * Z);
      d6[3] += val * (-X * Y);
      d6[4] += val * (-X * Z);
      d6[5] += val * (-Y * Z);
    }
  }
  for (int j = 0; j < 6; ++j) {
    sh[threadIdx.x] = d6[j];
    __syncthreads();
    for (int o = ADJ_T / 2; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) dsig_part[6 * blockIdx.x + j] = sh[0];
    __syncthreads();
  }
}

__global__ void __launch_bounds__(64) k_dsig_final(const double* __restrict__ part, int nblk, float* __restrict__ out) {
  __shared__ double sh[6][64];
  double a[6] = {0, 0, 0, 0, 0, 0};
  for (int i = threadIdx.x; i < nblk; i += 64)
    for (int j = 0; j < 6; ++j) a[j] += part[6 * i + j];
  for (int j = 0; j < 6; ++j) sh[j][threadIdx.x] = a[j];
  __syncthreads();
  if (threadIdx.x < 6) {
    double s = 0.0;
    for (int i = 0; i < 64; ++i) s += sh[threadIdx.x][i];
    out[threadIdx.x] = (float)s;
  }
}

// --------------------------------------------------------------- VJP sweep
// Sum over the 64 lanes of a wave in a fixed order (quads, half rows, rows,
// then row pairs, with DPP lane moves); the total ends in lane 63.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ float dpp_src(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWMASK, 0xF, false));
}
// Sum over each row of 16 lanes, left in every lane of the row.
__device__ __forceinline__ float row_sum(float v) {
  v += dpp_src<0xB1, 0xF>(v);    // quad_perm [1,0,3,2]
  v += dpp_src<0x4E, 0xF>(v);    // quad_perm [2,3,0,1]
  v += dpp_src<0x141, 0xF>(v);   // row_half_mirror
  v += dpp_src<0x140, 0xF>(v);   // row_mirror
  return v;
}

// Lane-per-entry gradient sweep.  A block owns n_sub consecutive entry chunks
// of vjp_chunk(MODE) band entries (in chunk g: wave w, step j, lane l -> entry
// 64 (w J + j) + l) and a range of at most VJP_TPB_MAX strip-ordered triangles,
// which are wave-uniform; the weighted phase factors of the two vertices a
// triangle shares with the previous one are carried over.  Pairs whose nodes
// are too close for the closed form are queued in LDS, one ring per stable
// scheme, and evaluated 64 at a time (vjp_lanes_pass), so each scheme runs on
// full waves instead of diverging.  Per triangle the lane sums
// are reduced over each row of 16 lanes (row_sum), over the rows and waves and
// then over the entry chunks, each in a fixed order, into part_out[NC][nt].
constexpr int VJP_TB = 32;   // triangles between block-level merges

// Queued pairs per wave and ring (power of two): at most 63 left from earlier
// triangles plus 64 J from the current one.
template <int J>
constexpr int vjp_ring() {
  return 64 + 64 * J <= 512 ? 512 : 1024;
}
static_assert(64 + 64 * VJP_J_MAX <= 1024, "ring too small");

// Two rings per wave: ring 0 holds pairs for the series (node spread below
// one radian), ring 1 pairs for the sorted scheme.  The fused sweep (FWD)
// keeps in fb the forward values of its queued pairs, one slot per entry, and
// writes each block's merged per-triangle sums straight out (its blocks own one
// entry chunk), so it has no per-block sum table.
template <int MODE, int J, bool FWD>
struct VjpLds {
  uint16_t queue[4][2][vjp_ring<J>()];
  float tot[4][4][VJP_TB][MODE == 0 ? 3 : 10];   // [wave][row of 16 lanes][triangle][channel]
  float sum[FWD ? 1 : VJP_TPB_MAX][MODE == 0 ? 3 : 10];
  float2 fb[4][FWD ? 64 * J : 1];   // [wave][entry offset 64 j + lane]
};

// Head, tail and end of the previous triangle's pairs in one ring.
struct VjpRing {
  int head, tail, prev_end;
};

// One gradient pair in closed form (caller checks the gaps, see LAG_GAP_RAD).
// Nodes z_p = -2 pi i t_p with t = (t1, t1 + a, t1 + b); with
// alpha = 1/(2 pi a), beta = 1/(2 pi b), gamma = 1/(2 pi (b - a)) the divided
// difference is the Lagrange sum T0 + T1 + T2,
//   T0 = -alpha beta E0,  T1 = alpha gamma E1,  T2 = -beta gamma E2   (E_p = e^{z_p}),
// and its derivatives in the nodes (the repeated-node DD4 of Eq. 10) are
//   DD4_0 = T0 + i[(alpha+beta) T0 + alpha T1 + beta T2]
//   DD4_1 = T1 + i[(gamma-alpha) T1 - alpha T0 + gamma T2]
//   DD4_2 = T2 - i[(beta+gamma) T2 + beta T0 + gamma T1].
// The adjoint weight enters through its modulus and phase, W E_p =
// |W| e^{-2 pi i (t_p - phi_W)}, so no complex product is formed.
//   VOLUME:  z[p] = Re(W DD4_p)          SURFACE: wf = Re(W f), z[p] = Im(W DD4_p)
// Closed-form gradient pair from the phase factors of the three nodes with
// the adjoint weight's phase folded in (G_p = e^{-2 pi i (t_p - phi_W)}) and
// the relative phases a, b in radians (2 pi times the a, b above).  With use false
// every output is exactly zero (the common factor 1 / (a b c) is replaced by
// zero, so a vanishing gap cannot produce inf or NaN).  With AMP
// the weight's modulus is folded into the Lagrange coefficients; without it
// the outputs are those of a unit modulus (the caller scales them) and
//   wf + i Pi = sum_p k_p G_p = e^{2 pi i phi_W} f_T,
// the forward value of the pair in the weight's phase frame.
//
// The Lagrange coefficients k0 = -1/(ab), k1 = 1/(ac), k2 = -1/(bc) are
// -c, b, -a times 1/(abc), and the node reciprocals follow from them:
// 1/a = c k1, 1/b = -a k0, 1/c = a k1.  Grouping the repeated-node terms by
// node pair, DD4_0 = T0 + i[(1/a)(T0 + T1) + (1/b)(T0 + T2)] and likewise for
// the other two nodes, so the three share the three pair sums.
template <int MODE, bool AMP>
__device__ __forceinline__ void lag_pair_g(float a, float b, bool use, float amp, float G0r, float G0i, float G1r,
                                           float G1i, float G2r, float G2i, float& wf, float z[3], float& Pi) {
  const float c = b - a;
  const float rD = use ? __builtin_amdgcn_rcpf(a * b * c) : 0.0f;   // 1 / (a b c), radians
  float k0, k1, k2, al, be, ga;
  if (AMP) {
    const float rw = amp * rD, k1u = b * rD;
    k0 = -c * rw;
    k1 = b * rw;
    k2 = -a * rw;
    al = c * k1u;
    ga = a * k1u;
    be = a * (c * rD);
  } else {
    k0 = -c * rD;
    k1 = b * rD;
    k2 = -a * rD;
    al = c * k1;
    be = -a * k0;
    ga = a * k1;
  }
  const float R0 = k0 * G0r, I0 = k0 * G0i, R1 = k1 * G1r, I1 = k1 * G1i, R2 = k2 * G2r, I2 = k2 * G2i;
  if (MODE == 0) {
    const float u01 = I0 + I1, u02 = I0 + I2, u12 = I1 + I2;
    z[0] = fmaf(-be, u02, fmaf(-al, u01, R0));
    z[1] = fmaf(-ga, u12, fmaf(al, u01, R1));
    z[2] = fmaf(ga, u12, fmaf(be, u02, R2));
    wf = R0 + R1 + R2;
    Pi = I0 + u12;
  } else {
    const float v01 = R0 + R1, v02 = R0 + R2, v12 = R1 + R2;
    z[0] = fmaf(be, v02, fmaf(al, v01, I0));
    z[1] = fmaf(ga, v12, fmaf(-al, v01, I1));
    z[2] = fmaf(-ga, v12, fmaf(-be, v02, I2));
    wf = R0 + v12;
    Pi = I0 + I1 + I2;
  }
}

// The gradient sweep folds the adjoint weight's modulus into the Lagrange
// coefficients where that is cheaper; the volume density and the fused sweep
// scale the outputs instead (the fused sweep needs the unscaled forward value).
template <int MODE, bool FWD>
constexpr bool vjp_amp_in_coeffs() {
  return MODE == 1 && !FWD;
}

// Closed-form pairs of one triangle: X holds the weighted phase factors of
// vertex 1, Y of vertex 2 (computed here at a strip start); on return X holds
// those of vertex 3, so the next triangle of the strip swaps X and Y.  Pairs
// that need the stable scheme are appended to the wave's ring of queued pairs
// (ring positions tail.., tagged with the triangle's parity).  The fused sweep
// (FWD) also adds the pair's forward value, weighted like the forward sweep's
// (k.n / L for the volume density, 2A for the surface density), to Fr + i Fi
// in the weight's phase frame.
template <int MODE, int J, bool FWD, bool OPQ>
__device__ __forceinline__ void vjp_lanes_main(const float* r, bool start, int tag, const float (&kx)[J],
                                               const float (&ky)[J], const float (&kz)[J], const float (&amp)[J],
                                               const float (&phw)[J], float (&Xr)[J], float (&Xi)[J], float (&Yr)[J],
                                               float (&Yi)[J], float (&Fr)[J], float (&Fi)[J], float tpx, float tpy,
                                               float tpz, int lane, uint16_t (*ring)[vjp_ring<J>()],
                                               VjpRing (&rq)[2], float (&acc)[MODE == 0 ? 3 : 10]) {
  constexpr bool AMP = vjp_amp_in_coeffs<MODE, FWD>();
  constexpr int NR = MODE == 0 ? (FWD ? 16 : 12) : 12;
  // the record in VGPRs: FP32 instructions with all operands in VGPRs issue
  // faster than those reading an SGPR, and vector loads of one address for
  // the whole wave (one cache line) cost no ALU slots, unlike per-value copies
  // from scalar registers; the zero made opaque keeps the loads vector loads
  float rvg[NR];
  if (MODE == 0) {
    int z = 0;
    asm volatile("" : "+v"(z));
    const float4* p4 = reinterpret_cast<const float4*>(r) + z;
#pragma unroll
    for (int i = 0; i < NR / 4; ++i) {
      const float4 q = p4[i];
      rvg[4 * i] = q.x;
      rvg[4 * i + 1] = q.y;
      rvg[4 * i + 2] = q.z;
      rvg[4 * i + 3] = q.w;
    }
  }
  const float* rv = MODE == 0 ? rvg : r;
  if (start) {
#pragma unroll
    for (int j = 0; j < J; ++j) {
      float d2, d3;
      rel_phases_rev(kx[j], ky[j], kz[j], rv, d2, d3);
      const float r1 = vertex3_phase(kx[j], ky[j], kz[j], rv) - d3 - phw[j];
      const float q1 = wrap(-r1), q2 = wrap(-(r1 + d2));
      Xr[j] = __builtin_amdgcn_cosf(q1);
      Xi[j] = __builtin_amdgcn_sinf(q1);
      Yr[j] = __builtin_amdgcn_cosf(q2);
      Yi[j] = __builtin_amdgcn_sinf(q2);
    }
  }
#pragma unroll
  for (int j = 0; j < J; ++j) {
    float a, b;
    rel_phases(kx[j], ky[j], kz[j], rv, a, b);
    const float q3 = vertex3_wphase(kx[j], ky[j], kz[j], rv, phw[j]);
    const float Nr = __builtin_amdgcn_cosf(q3), Ni = __builtin_amdgcn_sinf(q3);
    const float c = b - a;
    const float mn = fminf(fminf(fabsf(a), fabsf(b)), fabsf(c));
    const float mx = fmaxf(fmaxf(fabsf(a), fabsf(b)), fabsf(c));
    const bool close = mn < LAG_GAP_RAD, small = mx < SERIES_RAD && mn * mx < LAG_GAP_SPREAD;
    const bool fast = !close && !small;
    float wf = 0.0f, z[3], Pi;
    lag_pair_g<MODE, AMP>(a, b, fast, amp[j], Xr[j], Xi[j], Yr[j], Yi[j], Nr, Ni, wf, z, Pi);
    if (MODE == 0) {
#pragma unroll
      for (int p = 0; p < 3; ++p) acc[p] = fmaf(amp[j], z[p], acc[p]);
    } else {
      float x0 = kx[j] * tpx, x1 = ky[j] * tpy, x2 = kz[j] * tpz;
      if (AMP) {
        acc[0] += wf;
      } else {
        acc[0] = fmaf(amp[j], wf, acc[0]);
        x0 *= amp[j];
        x1 *= amp[j];
        x2 *= amp[j];
      }
#pragma unroll
      for (int p = 0; p < 3; ++p) {
        const float zp = z[p];
        acc[1 + 3 * p] = fmaf(zp, x0, acc[1 + 3 * p]);
        acc[2 + 3 * p] = fmaf(zp, x1, acc[2 + 3 * p]);
        acc[3 + 3 * p] = fmaf(zp, x2, acc[3 + 3 * p]);
      }
    }
    if (FWD) {
      const float wt = MODE == 0 ? fmaf(kz[j], rv[14], fmaf(ky[j], rv[13], kx[j] * rv[12])) : r[12];
      Fr[j] = fmaf(wt, wf, Fr[j]);
      Fi[j] = fmaf(wt, Pi, Fi[j]);
    }
    // Ballots of plain compares are the compares' own lane masks; the ballot
    // of the combined condition small would be rebuilt from a vector register
    // (two more instructions per pair), so its mask is the AND of its two
    // compares' ballots.  Lanes past the end of the band (all phases 0) are
    // queued too and skipped by the passes.
    const uint64_t bs =
        __builtin_amdgcn_ballot_w64(mx < SERIES_RAD) & __builtin_amdgcn_ballot_w64(mn * mx < LAG_GAP_SPREAD);
    const uint64_t bc = __builtin_amdgcn_ballot_w64(close) & ~bs;
    if (bs) {
      if (small) {
        const int pos = rq[0].tail + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bs >> 32),
                                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)bs, 0u));
        ring[0][pos & (vjp_ring<J>() - 1)] = OPQ ? queue_item(tag, j, lane) : plain_item(tag, j, lane);
      }
      rq[0].tail += __popcll(bs);
    }
    if (bc) {
      if (close && !small) {
        const int pos = rq[1].tail + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bc >> 32),
                                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)bc, 0u));
        ring[1][pos & (vjp_ring<J>() - 1)] = OPQ ? queue_item(tag, j, lane) : plain_item(tag, j, lane);
      }
      rq[1].tail += __popcll(bc);
    }
    Xr[j] = Nr;
    Xi[j] = Ni;
  }
}

// Stable scheme (KIND 0 series, 1 sorted) for n queued pairs from ring
// position head, on full waves: pairs tagged cur_tag belong to triangle r_cur
// (sums into acc_cur), the others to the previous triangle r_prev (acc_prev).
// erec_w points at the wave's first entry; n_w of its entries lie in the band
// (queued entries past them are skipped).  The fused sweep (FWD) adds each
// pair's weighted forward value to its entry's slot of fb, the pairs of the
// current triangle first, then those of the previous one (an entry is queued
// at most once per triangle), so no two lanes update one slot at once.
template <int MODE, int J, int KIND, bool FWD>
__device__ __forceinline__ void vjp_lanes_pass(const uint16_t* ring, int head, int n, const float* r_cur,
                                               const float* r_prev, int cur_tag, const float4* __restrict__ erec_w,
                                               int n_w, int lane, float (&acc_cur)[MODE == 0 ? 3 : 10],
                                               float (&acc_prev)[MODE == 0 ? 3 : 10], float2* fb) {
  constexpr int NC = MODE == 0 ? 3 : 10;
  wave_lds_sync();
  const int it = lane < n ? ring[(head + lane) & (vjp_ring<J>() - 1)] : 0;
  const int eo = 64 * ((it >> 6) & 7) + (it & 63);   // entry offset within the wave's 64 J
  float ffr = 0.0f, ffi = 0.0f;
  bool fact = false, fcur = false;
  if (lane < n && eo < n_w) {
    const bool cur = (it >> 9) == cur_tag;
    const float* r = cur ? r_cur : r_prev;
    const float4 A = erec_w[ERC * eo], B = erec_w[ERC * eo + 1];
    float tv, a, b, wf = 0.0f, z[3], fr, fi;
    tri_phases(A.x, A.y, A.z, r, tv, a, b);
    if (KIND == 0)
      vjp_pair_series<MODE>(tv, a, b, A.w, B.x, wf, z, fr, fi);
    else
      vjp_pair_sorted<MODE>(tv, a, b, A.w, B.x, wf, z, fr, fi);
    float add[NC];
    if (MODE == 0) {
#pragma unroll
      for (int p = 0; p < 3; ++p) add[p] = z[p];
    } else {
      add[0] = wf;
#pragma unroll
      for (int p = 0; p < 3; ++p) {
        add[1 + 3 * p] = z[p] * B.y;
        add[2 + 3 * p] = z[p] * B.z;
        add[3 + 3 * p] = z[p] * B.w;
      }
    }
#pragma unroll
    for (int ch = 0; ch < NC; ++ch) {
      acc_cur[ch] += cur ? add[ch] : 0.0f;
      acc_prev[ch] += cur ? 0.0f : add[ch];
    }
    if (FWD) {
      const float wt =
          MODE == 0 ? fmaf(A.z, r[14], fmaf(A.y, r[13], A.x * r[12])) : r[12];
      ffr = wt * fr;
      ffi = wt * fi;
      fact = true;
      fcur = cur;
    }
  }
  if (FWD) {
#pragma unroll
    for (int ph = 0; ph < 2; ++ph) {
      if (fact && fcur == (ph == 0)) {
        float2& s = fb[eo];
        s = make_float2(s.x + ffr, s.y + ffi);
      }
      wave_lds_sync();
    }
  }
}

// Row sums (16 lanes each) of one triangle into tot[w][row][tt]; the block
// merge adds the 4 rows of the 4 waves.
template <int MODE>
__device__ __forceinline__ void vjp_lanes_close(const float (&acc)[MODE == 0 ? 3 : 10], int tt, int lane, int w,
                                                float (*tot)[4][VJP_TB][MODE == 0 ? 3 : 10]) {
  constexpr int NC = MODE == 0 ? 3 : 10;
  float v[NC];
#pragma unroll
  for (int ch = 0; ch < NC; ++ch) v[ch] = row_sum(acc[ch]);
  // one store block, so the channels go out as wide LDS writes
  if ((lane & 15) == 0) {
#pragma unroll
    for (int ch = 0; ch < NC; ++ch) tot[w][lane >> 4][tt][ch] = v[ch];
  }
}

// Passes over ring KIND: full ones while 64 pairs are queued, then a partial
// one only if pairs of the previous triangle are still queued.
template <int MODE, int J, int KIND, bool FWD>
__device__ __forceinline__ void vjp_lanes_drain(VjpRing& q, const uint16_t* ring, bool prev_open, const float* r,
                                                const float* r_prev, int tag, const float4* __restrict__ erec_w,
                                                int n_w, int lane, float (&acc)[MODE == 0 ? 3 : 10],
                                                float (&acc_prev)[MODE == 0 ? 3 : 10], float2* fb) {
  while (q.tail - q.head >= 64) {
    vjp_lanes_pass<MODE, J, KIND, FWD>(ring, q.head, 64, r, r_prev, tag, erec_w, n_w, lane, acc, acc_prev, fb);
    q.head += 64;
  }
  if (prev_open && q.head < q.prev_end) {
    vjp_lanes_pass<MODE, J, KIND, FWD>(ring, q.head, q.tail - q.head, r, r_prev, tag, erec_w, n_w, lane, acc,
                                       acc_prev, fb);
    q.head = q.tail;
  }
}

// One triangle with the queue bookkeeping: full passes whenever 64 pairs are
// queued in a ring; the previous triangle (at most one other is open) is
// finished by partial passes only where some of its pairs are still queued, so
// most passes are full.  A triangle is closed (reduced into L.tot) once none
// of its pairs is queued in either ring.
template <int MODE, int J, bool FWD, bool OPQ>
__device__ __forceinline__ void vjp_lanes_step(const float* r, bool start, int tt, const float (&kx)[J],
                                               const float (&ky)[J], const float (&kz)[J], const float (&amp)[J],
                                               const float (&phw)[J], float (&Xr)[J], float (&Xi)[J], float (&Yr)[J],
                                               float (&Yi)[J], float (&Fr)[J], float (&Fi)[J],
                                               const float4* __restrict__ erec_w, int n_w, float tpx, float tpy,
                                               float tpz, int lane, int w, VjpLds<MODE, J, FWD>& L, VjpRing (&rq)[2],
                                               bool& prev_open, const float*& r_prev,
                                               float (&acc_prev)[MODE == 0 ? 3 : 10]) {
  constexpr int NC = MODE == 0 ? 3 : 10;
  // -0 is the additive identity (-0 + x == x for every x), so the first
  // additions fold away
  float acc[NC];
#pragma unroll
  for (int ch = 0; ch < NC; ++ch) acc[ch] = -0.0f;
  const int tag = tt & 1;
  vjp_lanes_main<MODE, J, FWD, OPQ>(r, start, tag, kx, ky, kz, amp, phw, Xr, Xi, Yr, Yi, Fr, Fi, tpx, tpy, tpz,
                                    lane, L.queue[w], rq, acc);
  vjp_lanes_drain<MODE, J, 0, FWD>(rq[0], L.queue[w][0], prev_open, r, r_prev, tag, erec_w, n_w, lane, acc, acc_prev,
                                   L.fb[w]);
  vjp_lanes_drain<MODE, J, 1, FWD>(rq[1], L.queue[w][1], prev_open, r, r_prev, tag, erec_w, n_w, lane, acc, acc_prev,
                                   L.fb[w]);
  if (prev_open) vjp_lanes_close<MODE>(acc_prev, tt - 1, lane, w, L.tot);
  if (rq[0].head == rq[0].tail && rq[1].head == rq[1].tail) {
    vjp_lanes_close<MODE>(acc, tt, lane, w, L.tot);
    prev_open = false;
  } else {
#pragma unroll
    for (int ch = 0; ch < NC; ++ch) acc_prev[ch] = acc[ch];
    prev_open = true;
    rq[0].prev_end = rq[0].tail;
    rq[1].prev_end = rq[1].tail;
    r_prev = r;
  }
}

// A block's tile: n_sub entry chunks of 256 J entries from e_begin times the
// strip-ordered triangles [t0, t1).  Gradient sweep (FWD false): the
// per-triangle sums of all its chunks are added in the block's sum table and
// written to part_out[NC][nt] at the end.  Fused sweep (FWD, n_sub = 1): they
// are written to part_out after every VJP_TB triangles, and each entry's
// forward sum over the tile, back in the plain phase frame and with the
// forward sweep's scaling, goes to fpart_row[entry].
template <int MODE, int J, bool FWD, bool OPQ = true>
__device__ __forceinline__ void vjp_lanes_tile(const float* __restrict__ rec, int nt, int t0, int t1,
                                               const float4* __restrict__ erec, int64_t nE, int64_t e_begin,
                                               int n_sub, float tpx, float tpy, float tpz,
                                               float* __restrict__ part_out, float2* __restrict__ fpart_row,
                                               VjpLds<MODE, J, FWD>& L) {
  constexpr int NC = MODE == 0 ? 3 : 10;
  // the wave index is wave-uniform: entry addresses get a scalar base
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (int g = 0; g < n_sub; ++g) {
    const int64_t ew = e_begin + (int64_t)g * 256 * J + (int64_t)w * 64 * J;
    const float4* erec_w = erec + ERC * ew;
    const int n_w = (int)max<int64_t>(0, min<int64_t>(nE - ew, 64 * J));   // entries of this wave in the band
    float kx[J], ky[J], kz[J], amp[J], phw[J];
    float Xr[J], Xi[J], Yr[J], Yi[J], Fr[J], Fi[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int64_t e = ew + 64 * j + lane;
      kx[j] = ky[j] = kz[j] = amp[j] = phw[j] = 0.0f;
      Xr[j] = Xi[j] = Yr[j] = Yi[j] = Fr[j] = Fi[j] = 0.0f;
      if (e < nE) {
        const float4 A = erec[ERC * e], C = erec[ERC * e + 2];
        kx[j] = A.x;
        ky[j] = A.y;
        kz[j] = A.z;
        amp[j] = C.x;
        phw[j] = C.y;
      }
      if (FWD) L.fb[w][64 * j + lane] = make_float2(0.0f, 0.0f);
    }
    for (int tb = t0; tb < t1; tb += VJP_TB) {
      const int tn = min(VJP_TB, t1 - tb);
      VjpRing rq[2] = {{0, 0, 0}, {0, 0, 0}};
      bool prev_open = false;
      const float* r_prev = rec + (size_t)tb * TRI_REC;
      float acc_prev[NC];
#pragma unroll
      for (int ch = 0; ch < NC; ++ch) acc_prev[ch] = 0.0f;
      for (int tt = 0; tt < tn; tt += 2) {
        const float* r = rec + (size_t)(tb + tt) * TRI_REC;
        vjp_lanes_step<MODE, J, FWD, OPQ>(r, tb + tt == t0 || r[15] != 0.0f, tt, kx, ky, kz, amp, phw, Xr, Xi, Yr,
                                          Yi, Fr, Fi, erec_w, n_w, tpx, tpy, tpz, lane, w, L, rq, prev_open, r_prev,
                                          acc_prev);
        if (tt + 1 < tn)
          vjp_lanes_step<MODE, J, FWD, OPQ>(r + TRI_REC, r[TRI_REC + 15] != 0.0f, tt + 1, kx, ky, kz, amp, phw, Yr,
                                            Yi, Xr, Xi, Fr, Fi, erec_w, n_w, tpx, tpy, tpz, lane, w, L, rq, prev_open,
                                            r_prev, acc_prev);
      }
      if (prev_open) {
        // only the last triangle (tn - 1) is still open: finish its pairs
        float none[NC];
#pragma unroll
        for (int ch = 0; ch < NC; ++ch) none[ch] = 0.0f;
        if (rq[0].tail > rq[0].head)
          vjp_lanes_pass<MODE, J, 0, FWD>(L.queue[w][0], rq[0].head, rq[0].tail - rq[0].head, r_prev, r_prev,
                                          (tn & 1), erec_w, n_w, lane, none, acc_prev, L.fb[w]);
        if (rq[1].tail > rq[1].head)
          vjp_lanes_pass<MODE, J, 1, FWD>(L.queue[w][1], rq[1].head, rq[1].tail - rq[1].head, r_prev, r_prev,
                                          (tn & 1), erec_w, n_w, lane, none, acc_prev, L.fb[w]);
        vjp_lanes_close<MODE>(acc_prev, tn - 1, lane, w, L.tot);
      }
      __syncthreads();
      for (int i = threadIdx.x; i < tn * NC; i += SWEEP_T) {
        const int tt = i / NC, ch = i - tt * NC;
        float v = 0.0f;
#pragma unroll
        for (int ww = 0; ww < 4; ++ww)
          v += (L.tot[ww][0][tt][ch] + L.tot[ww][1][tt][ch]) + (L.tot[ww][2][tt][ch] + L.tot[ww][3][tt][ch]);
        if (FWD) {
          part_out[(size_t)ch * nt + tb + tt] = v;
        } else {
          float& acc_t = L.sum[tb - t0 + tt][ch];
          acc_t = g == 0 ? v : acc_t + v;
        }
      }
      __syncthreads();
    }
    if (FWD) {
      // back from the weight's phase frame (multiply by e^{-2 pi i phi_W})
      wave_lds_sync();
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const int64_t e = ew + 64 * j + lane;
        if (e < nE) {
          const float q = wrap(phw[j]);
          const float cq = __builtin_amdgcn_cosf(q), sq = __builtin_amdgcn_sinf(q);
          const float ur = fmaf(Fr[j], cq, Fi[j] * sq), ui = fmaf(Fi[j], cq, -Fr[j] * sq);
          const float2 qb = L.fb[w][64 * j + lane];
          fpart_row[e] = make_float2(ur + qb.x, ui + qb.y);
        }
      }
    }
  }
  if (!FWD) {
    for (int i = threadIdx.x; i < (t1 - t0) * NC; i += SWEEP_T) {
      const int tl = i / NC, ch = i - tl * NC;
      part_out[(size_t)ch * nt + t0 + tl] = n_sub > 0 ? L.sum[tl][ch] : 0.0f;
    }
  }
}

// At most 96 VGPRs in volume mode (5 waves per SIMD; one more register
// granule would leave 4) and 128 in surface mode (4 waves, with 6 entries per
// lane: 8 entries needed about 150 registers, 3 waves, and ran 4% slower).
template <int MODE>
__global__ void __launch_bounds__(SWEEP_T, MODE == 0 ? 5 : 4) k_vjp_lanes(GridC g, const float* __restrict__ rec, int nt, int tpb,
                                                         const float4* __restrict__ erec, int64_t nE, int n_sub,
                                                         float* __restrict__ part) {
  constexpr int J = vjp_j(MODE);
  __shared__ VjpLds<MODE, J, false> L;
  constexpr int NC = MODE == 0 ? 3 : 10;
  const int t0 = blockIdx.y * tpb;
  const int64_t e_begin = (int64_t)blockIdx.x * n_sub * vjp_chunk(MODE);
  const int sub = (int)min<int64_t>(n_sub, (nE - e_begin + vjp_chunk(MODE) - 1) / vjp_chunk(MODE));
  vjp_lanes_tile<MODE, J, false>(rec, nt, t0, min(nt, t0 + tpb), erec, nE, e_begin, sub, g.two_pi_over_L[0],
                                 g.two_pi_over_L[1], g.two_pi_over_L[2], part + (size_t)blockIdx.x * NC * nt, nullptr,
                                 L);
}

// Fused forward and gradient sweep for a given cotangent: one entry chunk of
// fused_chunk(MODE) entries per block (blockIdx.x) times a range of tpb
// triangles (blockIdx.y).  Writes the gradient partials part[x][NC][nt] like
// k_vjp_lanes and the forward partials fpart[y][nE] like k_fwd_lanes.  Same
// register budgets as the gradient sweep (one entry per lane fewer).
constexpr int FUSED_WAVES_VOLUME = 4, FUSED_WAVES_SURFACE = 4;
template <int MODE>
__global__ void __launch_bounds__(SWEEP_T, MODE == 0 ? FUSED_WAVES_VOLUME : FUSED_WAVES_SURFACE)
    k_fused_lanes(GridC g, const float* __restrict__ rec, int nt, int tpb, const float4* __restrict__ erec,
                  int64_t nE, float* __restrict__ part, float2* __restrict__ fpart) {
  constexpr int J = fused_j(MODE);
  __shared__ VjpLds<MODE, J, true> L;
  constexpr int NC = MODE == 0 ? 3 : 10;
  const int t0 = blockIdx.y * tpb;
  const int64_t e_begin = (int64_t)blockIdx.x * fused_chunk(MODE);
  vjp_lanes_tile<MODE, J, true>(rec, nt, t0, min(nt, t0 + tpb), erec, nE, e_begin, 1, g.two_pi_over_L[0],
                                g.two_pi_over_L[1], g.two_pi_over_L[2], part + (size_t)blockIdx.x * NC * nt,
                                fpart + (size_t)blockIdx.y * nE, L);
}

// Persistent sweeps over the work items of many independent meshes: one
// launch per kind of tile (forward or gradient) and density mode, since their
// register and LDS footprints differ and each should run at its own occupancy.  Each
// workgroup takes the next item from a global counter; every item writes its
// own partial slot, so the results do not depend on which workgroup ran which
// item.
// Work items and requests are read after the sweeps' stores, so the compiler
// cannot keep them in scalar registers by itself; they are wave-uniform, and
// these copies say so (otherwise they occupy vector registers in the sweeps).
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ float uni(float x) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x))); }
template <typename T>
__device__ __forceinline__ T* uni(T* p) {
  const uint64_t v = (uint64_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v), hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (T*)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ SweepItem uni(const SweepItem& w) { return {uni(w.kind), uni(w.req), uni(w.x0), uni(w.c)}; }
__device__ __forceinline__ SweepReq uni(const SweepReq& q) {
  SweepReq u;
  u.mode = uni(q.mode);
  u.nE = uni(q.nE);
  u.nt = uni(q.nt);
  u.tpc = uni(q.tpc);
  u.epc = uni(q.epc);
  u.vsub = uni(q.vsub);
  u.vtpb = uni(q.vtpb);
  u.tile0 = uni(q.tile0);
  u.tpx = uni(q.tpx);
  u.tpy = uni(q.tpy);
  u.tpz = uni(q.tpz);
  u.ntr = uni(q.ntr);
  u.kf = uni(q.kf);
  u.rec = uni(q.rec);
  u.fpart = uni(q.fpart);
  u.erec = uni(q.erec);
  u.vpart = uni(q.vpart);
  return u;
}

__device__ __forceinline__ int next_item(int* counter, int* slot) {
  if (threadIdx.x == 0) *slot = atomicAdd(counter, 1);
  __syncthreads();
  const int it = __builtin_amdgcn_readfirstlane(*slot);
  __syncthreads();
  return it;
}

template <int MODE>
__global__ void __launch_bounds__(SWEEP_T, 7) k_batch_fwd(const SweepItem* __restrict__ items, int n_items,
                                                         const SweepReq* __restrict__ reqs, int* __restrict__ counter) {
  __shared__ int slot;
  __shared__ FwdLds L;
  for (;;) {
    const int it = next_item(counter, &slot);
    if (it >= n_items) return;
    const SweepItem w = uni(items[it]);
    const SweepReq q = uni(reqs[w.req]);
    const int t0 = w.c * q.tpc, t1 = min(q.nt, t0 + q.tpc);
    fwd_lanes_tile<MODE>(q.kf, q.nE, q.rec, t0, t1, w.x0, q.fpart + (size_t)w.c * q.nE, L);
  }
}

// The item loop around the tile must not cost occupancy: at least as many
// waves per SIMD as the single-request gradient sweep (5 volume, 4 surface).
template <int MODE>
__global__ void __launch_bounds__(SWEEP_T, MODE == 0 ? 5 : 4)
    k_batch_vjp(const SweepItem* __restrict__ items, int n_items, const SweepReq* __restrict__ reqs,
                int* __restrict__ counter) {
  constexpr int NC = MODE == 0 ? 3 : 10;
  constexpr int J = vjp_j(MODE);
  __shared__ int slot;
  __shared__ VjpLds<MODE, J, false> L;
  for (;;) {
    const int it = next_item(counter, &slot);
    if (it >= n_items) return;
    const SweepItem w = uni(items[it]);
    const SweepReq q = uni(reqs[w.req]);
    const int64_t e_begin = (int64_t)w.c * q.epc;
    const int sub = (int)min<int64_t>(q.vsub, ((int64_t)q.nE - e_begin + vjp_chunk(MODE) - 1) / vjp_chunk(MODE));
    const int t1 = min(q.nt, w.x0 + q.vtpb);
    vjp_lanes_tile<MODE, J, false, MODE == 0>(q.rec, q.nt, w.x0, t1, q.erec, q.nE, e_begin, sub, q.tpx, q.tpy,
                                              q.tpz, q.vpart + (size_t)w.c * NC * q.nt, nullptr, L);
  }
}

// Persistent fused sweep (forward and gradient) over the tiles of many
// requests: tile t of request r (t counted from its tile0) is entry chunk
// t / ntr and triangle range t % ntr, so each request's partials have the
// layout of k_fused_lanes with its own triangle ranges.  Workgroups take the
// next tile from a counter; tiles come in increasing order, so a workgroup
// finds its request by advancing from the previous one.
template <int MODE>
__global__ void __launch_bounds__(SWEEP_T, MODE == 0 ? FUSED_WAVES_VOLUME : FUSED_WAVES_SURFACE)
    k_batch_fused(const SweepReq* __restrict__ reqs, int n_reqs, int n_tiles, int* __restrict__ counter) {
  constexpr int NC = MODE == 0 ? 3 : 10;
  constexpr int J = fused_j(MODE);
  __shared__ int slot;
  __shared__ VjpLds<MODE, J, true> L;
  int r = 0;
  for (;;) {
    const int tile = next_item(counter, &slot);
    if (tile >= n_tiles) return;
    while (r + 1 < n_reqs && tile >= uni(reqs[r + 1].tile0)) ++r;
    const SweepReq q = uni(reqs[r]);
    const int local = tile - q.tile0;
    const int c = local / q.ntr, y = local - c * q.ntr;
    const int t0 = y * q.vtpb, t1 = min(q.nt, t0 + q.vtpb);
    vjp_lanes_tile<MODE, J, true, MODE == 0>(q.rec, q.nt, t0, t1, q.erec, q.nE, (int64_t)c * fused_chunk(MODE), 1,
                                             q.tpx, q.tpy,
                                  q.tpz, q.vpart + (size_t)c * NC * q.nt, q.fpart + (size_t)y * q.nE, L);
  }
}

// Split reduction of the gradient partials in two fixed-order levels:
// group g sums chunks [g*per, (g+1)*per), then the groups are summed in order.
__global__ void k_vjp_reduce_groups(const float* __restrict__ part, int n_chunks, int per, int64_t n,
                                    float* __restrict__ tmp) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c0 = blockIdx.y * per, c1 = min(n_chunks, c0 + per);
  float s = 0.0f;
  for (int c = c0; c < c1; ++c) s += part[(size_t)c * n + i];
  tmp[(size_t)blockIdx.y * n + i] = s;
}

__global__ void k_vjp_reduce_final(const float* __restrict__ tmp, int groups, int64_t n, float* __restrict__ red) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = 0.0f;
  for (int g = 0; g < groups; ++g) s += tmp[(size_t)g * n + i];
  red[i] = s;
}

// R = (1/|Lambda|) sum_T 2 A_T s_T  (surface normalisation term of Eq. 6; with density
// weights the record carries w_T 2 A_T and |Lambda| is sum_T w_T A_T)
__global__ void __launch_bounds__(PREP_T) k_surface_scalar(const float* __restrict__ red,
                                                             const float* __restrict__ rec, int nt,
                                                             const MeshInfo* __restrict__ info,
                                                             double* __restrict__ out) {
  __shared__ double sh[PREP_T];
  double a = 0.0;
  for (int t = threadIdx.x; t < nt; t += PREP_T) a += (double)rec[(size_t)t * TRI_REC + 12] * (double)red[t];
  a = block_sum(a, sh);
  if (threadIdx.x == 0) *out = a / info->area;
}

template <int MODE>
__global__ void k_vertex_gather(const float* __restrict__ V, int nv, const int32_t* __restrict__ F,
                                const int32_t* __restrict__ flags, const float* __restrict__ tri_w, int nt,
                                const int32_t* __restrict__ off, const int32_t* __restrict__ ent,
                                const float* __restrict__ red, const double* __restrict__ Rp,
                                float* __restrict__ dV) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  const float R = MODE == 1 ? (float)(*Rp) : 0.0f;
  float g[3] = {0.0f, 0.0f, 0.0f};
  for (int i = off[v]; i < off[v + 1]; ++i) {
    const int tp = ent[i];
    const int t = tp / 3, p = tp - 3 * t;
    const float wt = tri_w != nullptr ? tri_w[t] : 1.0f;
    float x[3][3];
    for (int q = 0; q < 3; ++q) {
      const int vi = F[3 * t + q];
      for (int j = 0; j < 3; ++j) x[q][j] = V[3 * vi + j];
    }
    const float a[3] = {x[1][0] - x[0][0], x[1][1] - x[0][1], x[1][2] - x[0][2]};
    const float b[3] = {x[2][0] - x[0][0], x[2][1] - x[0][1], x[2][2] - x[0][2]};
    const float n[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
    if (MODE == 0) {
      const float Qs = (flags[t] & TRI_REVERSED) ? -red[(size_t)p * nt + t] : red[(size_t)p * nt + t];
      const float Q = wt * Qs;
      for (int j = 0; j < 3; ++j) g[j] = fmaf(n[j], Q, g[j]);
    } else {
      const float twoA = sqrtf(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
      const float inv = twoA > 0.0f ? 1.0f / twoA : 0.0f;
      const float N[3] = {n[0] * inv, n[1] * inv, n[2] * inv};
      const int pm = (p + 2) % 3, pp = (p + 1) % 3;
      const float ep[3] = {x[pm][0] - x[pp][0], x[pm][1] - x[pp][1], x[pm][2] - x[pp][2]};
      const float w[3] = {ep[1] * N[2] - ep[2] * N[1], ep[2] * N[0] - ep[0] * N[2], ep[0] * N[1] - ep[1] * N[0]};
      const float s = red[t];
      for (int j = 0; j < 3; ++j) {
        const float P = red[(size_t)(1 + 3 * p + j) * nt + t];
        g[j] += wt * (twoA * P - w[j] * s + 0.5f * R * w[j]);
      }
    }
  }
  for (int j = 0; j < 3; ++j) dV[3 * v + j] = g[j];
}

// ------------------------------------------------------ arbitrary points
__global__ void k_points_prepare(const int32_t* __restrict__ k, int64_t n, float4* __restrict__ kf) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  kf[i] = make_float4((float)k[3 * i], (float)k[3 * i + 1], (float)k[3 * i + 2], 1.0f);
}

template <int MODE>
__global__ void k_points_finalize(GridC g, const float4* __restrict__ kf, int64_t n, const float2* __restrict__ part,
                                  int n_chunks, const MeshInfo* __restrict__ info, float2* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float sr = 0.0f, si = 0.0f;
  for (int c = 0; c < n_chunks; ++c) {
    const float2 v = part[(size_t)c * n + i];
    sr += v.x;
    si += v.y;
  }
  const float4 k = kf[i];
  out[i] = finish_u<MODE>(g, info, k.x, k.y, k.z, sr, si);
}

__global__ void k_fill_zero(float* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0f;
}

inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

// ------------------------------------------------------------- launchers
hipError_t launch_fill_zero(float* p, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_zero, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_band_count(const GridC& g, const double* sigma6, double qmax, int32_t* cnt, int64_t n_slots,
                             hipStream_t s) {
  Sig6 S;
  for (int j = 0; j < 6; ++j) S.s[j] = sigma6[j];
  hipLaunchKernelGGL(k_band_count, dim3(blocks_for(n_slots, 256)), dim3(256), 0, s, g, S, qmax, cnt, n_slots);
  return hipGetLastError();
}

int64_t scan_tmp_elems(int64_t n) { return (n + SCAN_BLK - 1) / SCAN_BLK + 1; }

hipError_t launch_scan(const int32_t* in, int32_t* out, int64_t n, int32_t* block_tmp, int64_t* total,
                       hipStream_t s) {
  const int64_t nb = (n + SCAN_BLK - 1) / SCAN_BLK;
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(SCAN_T), 0, s, in, n, block_tmp);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(SCAN_T), 0, s, block_tmp, nb, total);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(SCAN_T), 0, s, in, out, n, (const int32_t*)block_tmp);
  return hipGetLastError();
}

hipError_t launch_band_fill(const GridC& g, const double* sigma6, double qmax, const int32_t* cnt,
                            const int32_t* off, int64_t n_slots, BandDev b, hipStream_t s) {
  Sig6 S;
  for (int j = 0; j < 6; ++j) S.s[j] = sigma6[j];
  hipLaunchKernelGGL(k_band_fill, dim3(blocks_for(n_slots, 256)), dim3(256), 0, s, g, S, qmax, cnt, off, n_slots, b);
  return hipGetLastError();
}

hipError_t launch_band_count_otf(const GridC& g, const float2* otf, double tau2, int32_t* cnt, int64_t n_slots,
                                 hipStream_t s) {
  hipLaunchKernelGGL(k_band_count_otf, dim3(blocks_for(n_slots, 256)), dim3(256), 0, s, g, otf, tau2, cnt, n_slots);
  return hipGetLastError();
}

hipError_t launch_band_fill_otf(const GridC& g, const float2* otf, double tau2, const int32_t* cnt,
                                const int32_t* off, int64_t n_slots, BandDev b, hipStream_t s) {
  hipLaunchKernelGGL(k_band_fill_otf, dim3(blocks_for(n_slots, 256)), dim3(256), 0, s, g, otf, tau2, cnt, off,
                     n_slots, b);
  return hipGetLastError();
}

int mesh_prep_blocks(int nt) {
  int b = (nt + PREP_T - 1) / PREP_T;
  return b < 1 ? 1 : (b > 1024 ? 1024 : b);
}

hipError_t launch_mesh_prep(int mode, const GridC& g, const float* verts, int nv, const int32_t* faces,
                            const int32_t* flags, const float* tri_w, int nt,
                            float* tri_rec, MeshInfo* info, double* block_tmp, int tmp_blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_prep_centroid, dim3(1), dim3(PREP_T), 0, s, g, verts, nv, info);
  if (mode == 0)
    hipLaunchKernelGGL(k_prep_tris<0>, dim3(tmp_blocks), dim3(PREP_T), 0, s, g, verts, faces, flags, tri_w, nt,
                       (const MeshInfo*)info, tri_rec, block_tmp);
  else
    hipLaunchKernelGGL(k_prep_tris<1>, dim3(tmp_blocks), dim3(PREP_T), 0, s, g, verts, faces, flags, tri_w, nt,
                       (const MeshInfo*)info, tri_rec, block_tmp);
  hipLaunchKernelGGL(k_prep_totals, dim3(1), dim3(PREP_T), 0, s, (const double*)block_tmp, tmp_blocks, info);
  return hipGetLastError();
}

hipError_t launch_fwd_lanes(int mode, const float4* kf, int64_t nE, const float* tri_rec, int nt, int tris_per_chunk,
                            int n_chunks, float2* part, hipStream_t s) {
  if (tris_per_chunk < 1 || (int64_t)tris_per_chunk * n_chunks < nt) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((nE + FWD_CHUNK - 1) / FWD_CHUNK), (unsigned)n_chunks);
  if (mode == 0)
    hipLaunchKernelGGL(k_fwd_lanes<0>, grid, dim3(SWEEP_T), 0, s, kf, nE, tri_rec, nt, tris_per_chunk, part);
  else
    hipLaunchKernelGGL(k_fwd_lanes<1>, grid, dim3(SWEEP_T), 0, s, kf, nE, tri_rec, nt, tris_per_chunk, part);
  return hipGetLastError();
}


hipError_t launch_fwd_finalize(int mode, const GridC& g, BandDev b, const float2* part, int n_chunks,
                               const MeshInfo* info, float2* spec_out, float2* xhalf, hipStream_t s) {
  const dim3 grid(blocks_for(b.n_pos, 256));
  if (mode == 0)
    hipLaunchKernelGGL(k_fwd_finalize<0>, grid, dim3(256), 0, s, g, b, part, n_chunks, info, spec_out, xhalf);
  else
    hipLaunchKernelGGL(k_fwd_finalize<1>, grid, dim3(256), 0, s, g, b, part, n_chunks, info, spec_out, xhalf);
  return hipGetLastError();
}

hipError_t launch_spec_scatter(const GridC& g, BandDev b, const float2* spec, float2* xhalf, hipStream_t s) {
  hipLaunchKernelGGL(k_spec_scatter, dim3(blocks_for(b.n_pos, 256)), dim3(256), 0, s, g, b, spec, xhalf);
  return hipGetLastError();
}

int adjoint_blocks(const GridC& g) {
  const int64_t npos = (int64_t)g.n0 * g.n1 * g.n2h;
  int64_t b = (npos + ADJ_T - 1) / ADJ_T;
  if (b > 2048) b = 2048;
  return (int)(b < 1 ? 1 : b);
}

hipError_t launch_adjoint(int mode, const GridC& g, BandDev b, const float2* ghat, const MeshInfo* info, float4* erec,
                          hipStream_t s) {
  const dim3 grid(blocks_for(b.n_pos, 256));
  if (mode == 0)
    hipLaunchKernelGGL(k_adjoint<0>, grid, dim3(256), 0, s, g, b, ghat, info, erec);
  else
    hipLaunchKernelGGL(k_adjoint<1>, grid, dim3(256), 0, s, g, b, ghat, info, erec);
  return hipGetLastError();
}

hipError_t launch_dsig(const GridC& g, BandDev b, const float2* ghat, const float2* spec, double* dsig_part,
                       int dsig_blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_dsig, dim3(dsig_blocks), dim3(ADJ_T), 0, s, g, b, ghat, spec, dsig_part);
  return hipGetLastError();
}

hipError_t launch_dsig_final(const double* dsig_part, int nblk, float* out6, hipStream_t s) {
  hipLaunchKernelGGL(k_dsig_final, dim3(1), dim3(64), 0, s, dsig_part, nblk, out6);
  return hipGetLastError();
}

hipError_t launch_batch_sweep(const SweepItem* items, const int* group_end, const SweepReq* reqs,
                              const SweepReq* const* fused_reqs, const int* n_fused_reqs, const int* n_fused_tiles,
                              int* counters, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_zero, dim3(1), dim3(64), 0, s, reinterpret_cast<float*>(counters),
                     (int64_t)BATCH_GROUPS);
  const dim3 threads(SWEEP_T);
  int begin = 0;
  for (int grp = 0; grp < 4; ++grp) {
    const int n = group_end[grp] - begin;
    if (n > 0) {
      const SweepItem* it = items + begin;
      // one resident round of workgroups (4 waves each) at the kernel's occupancy
      const dim3 blocks((unsigned)std::min(n, grp < 2 ? 2048 : 1280));
      if (grp == 0) hipLaunchKernelGGL(k_batch_fwd<0>, blocks, threads, 0, s, it, n, reqs, counters);
      if (grp == 1) hipLaunchKernelGGL(k_batch_fwd<1>, blocks, threads, 0, s, it, n, reqs, counters + 1);
      if (grp == 2) hipLaunchKernelGGL(k_batch_vjp<0>, blocks, threads, 0, s, it, n, reqs, counters + 2);
      if (grp == 3) hipLaunchKernelGGL(k_batch_vjp<1>, blocks, threads, 0, s, it, n, reqs, counters + 3);
    }
    begin = group_end[grp];
  }
  for (int m = 0; m < 2; ++m) {
    const int n = n_fused_tiles[m];
    if (n <= 0 || n_fused_reqs[m] <= 0) continue;
    const dim3 blocks((unsigned)std::min(n, 1024));   // 4 waves per SIMD: 4 workgroups per CU
    if (m == 0)
      hipLaunchKernelGGL(k_batch_fused<0>, blocks, threads, 0, s, fused_reqs[0], n_fused_reqs[0], n, counters + 4);
    else
      hipLaunchKernelGGL(k_batch_fused<1>, blocks, threads, 0, s, fused_reqs[1], n_fused_reqs[1], n, counters + 5);
  }
  return hipGetLastError();
}

hipError_t launch_vjp_lanes(int mode, const GridC& g, const float* tri_rec, int nt, int tris_per_block,
                            int chunks_per_block, int n_chunks, const float4* erec, int64_t nE, float* part,
                            hipStream_t s) {
  if (tris_per_block < 1 || tris_per_block > VJP_TPB_MAX || chunks_per_block < 1 ||
      (int64_t)n_chunks * chunks_per_block * vjp_chunk(mode) < nE)
    return hipErrorInvalidValue;
  const dim3 grid((unsigned)n_chunks, blocks_for(nt, tris_per_block));
  if (mode == 0)
    hipLaunchKernelGGL(k_vjp_lanes<0>, grid, dim3(SWEEP_T), 0, s, g, tri_rec, nt, tris_per_block, erec, nE,
                       chunks_per_block, part);
  else
    hipLaunchKernelGGL(k_vjp_lanes<1>, grid, dim3(SWEEP_T), 0, s, g, tri_rec, nt, tris_per_block, erec, nE,
                       chunks_per_block, part);
  return hipGetLastError();
}

hipError_t launch_fused_lanes(int mode, const GridC& g, const float* tri_rec, int nt, int tris_per_block,
                              const float4* erec, int64_t nE, float* part, float2* fpart, hipStream_t s) {
  if (tris_per_block < 1 || nE < 1 || nt < 1) return hipErrorInvalidValue;
  const dim3 grid(blocks_for(nE, fused_chunk(mode)), blocks_for(nt, tris_per_block));
  if (mode == 0)
    hipLaunchKernelGGL(k_fused_lanes<0>, grid, dim3(SWEEP_T), 0, s, g, tri_rec, nt, tris_per_block, erec, nE, part,
                       fpart);
  else
    hipLaunchKernelGGL(k_fused_lanes<1>, grid, dim3(SWEEP_T), 0, s, g, tri_rec, nt, tris_per_block, erec, nE, part,
                       fpart);
  return hipGetLastError();
}

int vjp_reduce_groups(int n_chunks) { return n_chunks < 32 ? n_chunks : 32; }

hipError_t launch_vjp_reduce(int mode, const float* part, int n_chunks, int nt, float* tmp, float* red,
                             hipStream_t s) {
  const int64_t n = (int64_t)nchannels(mode) * nt;
  const int groups = vjp_reduce_groups(n_chunks);
  const int per = (n_chunks + groups - 1) / groups;
  const int used = (n_chunks + per - 1) / per;
  hipLaunchKernelGGL(k_vjp_reduce_groups, dim3(blocks_for(n, 256), (unsigned)used), dim3(256), 0, s, part, n_chunks,
                     per, n, tmp);
  hipLaunchKernelGGL(k_vjp_reduce_final, dim3(blocks_for(n, 256)), dim3(256), 0, s, (const float*)tmp, used, n, red);
  return hipGetLastError();
}

hipError_t launch_surface_scalar(const float* red, const float* tri_rec, int nt, const MeshInfo* info,
                                 double* out_R, hipStream_t s) {
  hipLaunchKernelGGL(k_surface_scalar, dim3(1), dim3(PREP_T), 0, s, red, tri_rec, nt, info, out_R);
  return hipGetLastError();
}

hipError_t launch_vertex_gather(int mode, const float* verts, int nv, const int32_t* faces, const int32_t* flags,
                                const float* tri_w, int nt,
                                const int32_t* csr_off, const int32_t* csr_ent, const float* red,
                                const double* R, float* dV, hipStream_t s) {
  const dim3 grid(blocks_for(nv, 128));
  if (mode == 0)
    hipLaunchKernelGGL(k_vertex_gather<0>, grid, dim3(128), 0, s, verts, nv, faces, flags, tri_w, nt, csr_off, csr_ent,
                       red, R, dV);
  else
    hipLaunchKernelGGL(k_vertex_gather<1>, grid, dim3(128), 0, s, verts, nv, faces, flags, tri_w, nt, csr_off, csr_ent,
                       red, R, dV);
  return hipGetLastError();
}

hipError_t launch_points_prepare(const GridC& g, const int32_t* k, int64_t n, float4* kf, hipStream_t s) {
  (void)g;
  hipLaunchKernelGGL(k_points_prepare, dim3(blocks_for(n, 256)), dim3(256), 0, s, k, n, kf);
  return hipGetLastError();
}

hipError_t launch_points_finalize(int mode, const GridC& g, const float4* kf, int64_t n, const float2* part,
                                  int n_chunks, const MeshInfo* info, float2* out, hipStream_t s) {
  if (mode == 0)
    hipLaunchKernelGGL(k_points_finalize<0>, dim3(blocks_for(n, 256)), dim3(256), 0, s, g, kf, n, part, n_chunks, info,
                       out);
  else
    hipLaunchKernelGGL(k_points_finalize<1>, dim3(blocks_for(n, 256)), dim3(256), 0, s, g, kf, n, part, n_chunks, info,
                       out);
  return hipGetLastError();
}

}  // namespace dm

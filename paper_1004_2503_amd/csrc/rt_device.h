// rt_device.h -- device-side building blocks shared by the gfx950 kernels of
// librt_m1.so: fast math helpers, the M1 closure (Sec. 2.2), the hydrogen
// rate set and the sub-cycled per-cell chemistry operator Phi (Sec. 2.2,
// Appendix A).  Included by the step kernel, the batch chemistry kernel and
// the surrogate kernels.
#pragma once

#include <math.h>

#include "rt_internal.h"

namespace rtk {

// ------------------------------------------------------------ math helpers
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double frcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double fsqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float fexp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float flog2(float x) { return __builtin_amdgcn_logf(x); }
template <typename R> __device__ __forceinline__ R rmin(R a, R b) { return a < b ? a : b; }
template <typename R> __device__ __forceinline__ R rmax(R a, R b) { return a > b ? a : b; }

// --------------------------------------------------- M1 closure (Sec. 2.2)
// P = D N, D = (1-chi)/2 I + (3chi-1)/2 n(x)n, chi(f) of Levermore with
// f = |F|/(cN) clamped to [0, 1], evaluated on the reduced flux u = F/(cN).
struct Press {
    float xx, yy, zz, xy, xz, yz;
};

// Radiation densities below N_TINY are treated as empty: their reciprocals
// would leave the normal FP32 range.
constexpr float N_TINY = 1e-30f;

// P = D N, times ns (the HLL step keeps c^2 P, the physical flux of F,
// so that no face multiplies by c^2 again; ns = 1 gives P itself)
__device__ __forceinline__ Press closure(float N, float Fx, float Fy, float Fz,
                                         float inv_c, float ns = 1.0f)
{
    Press P;
    if (!(N > N_TINY)) {
        P.xx = P.yy = P.zz = P.xy = P.xz = P.yz = 0.0f;
        return P;
    }
    // reduced flux u = F/(cN), |u| = f
    const float s = inv_c * frcp(N);
    const float ux = Fx * s, uy = Fy * s, uz = Fz * s;
    const float u2 = ux * ux + uy * uy + uz * uz;
    const float f2 = rmin(u2, 1.0f);
    const float chi = (3.0f + 4.0f * f2) * frcp(5.0f + 2.0f * fsqrt(4.0f - 3.0f * f2));
    const float Ns = N * ns;
    const float iso = 0.5f * (1.0f - chi) * Ns;
    // (3chi-1)/2 N n_i n_j with n = u/|u|; negligible below f^2 = 1e-30
    const float w = (u2 > 1e-30f) ? 0.5f * (3.0f * chi - 1.0f) * Ns * frcp(u2) : 0.0f;
    P.xx = iso + w * ux * ux;
    P.yy = iso + w * uy * uy;
    P.zz = iso + w * uz * uz;
    P.xy = w * ux * uy;
    P.xz = w * ux * uz;
    P.yz = w * uy * uz;
    return P;
}

// ------------------------------------------------- HLL signal speeds
// Sec. 2.2 names HLL beside LF.  Its speeds are c times the smallest and
// largest eigenvalue of the M1 flux Jacobian along an axis.  With f the
// reduced flux, mu the cosine of its angle to the axis and S =
// sqrt(4 - 3 f^2), the characteristic polynomial factors as
// (lambda - m)^2 (lambda^2 - B lambda + C), B = mu chi'(f), so that
//   lambda = (B -+ sqrt(B^2 - 4C)) / 2,
//   B^2 - 4C = 8 (S-1) [(S-1)(1+mu^2) + (1-mu^2)] / (3 S^2),
//   S - 1 = 3 (1 - f^2) / (S + 1):
// every factor is a sum of non-negative terms, so nothing cancels near free
// streaming, where both speeds tend to mu.  1 - f^2 is formed in FP64 from
// the FP32 state; 1 - mu^2 from the other two flux components.  Empty cells
// take the isotropic speeds -+1/sqrt(3).
struct Speeds {
    float xm, xp, ym, yp, zm, zp;
};

// The parts of the eigenvalue formula shared by the three axes.
struct SpeedPrep {
    bool iso;                       // isotropic (no flux): -+1/sqrt(3) on every axis
    float ux, uy, uz, x2, y2, z2, inv_f2, pref, Sm1, Q;
};

// The extreme eigenvalues along one axis: ud the reduced flux along it, a2
// its square, o2 the sum of the other two squares.
__device__ __forceinline__ void m1_axis(const SpeedPrep &p, float ud, float a2, float o2,
                                        float &lm, float &lp)
{
    if (p.iso) {
        lm = -0.5773502691896258f;
        lp = 0.5773502691896258f;
        return;
    }
    const float r = fsqrt(p.pref * (p.Sm1 * (1.0f + a2 * p.inv_f2) + o2 * p.inv_f2));
    const float B = ud * p.Q;
    lm = 0.5f * (B - r);
    lp = 0.5f * (B + r);
}

// The HLL form needs both the pressure (times ns) and the parts of the
// speed formula shared by the three axes: one pass shares 1/N, the reduced
// flux, 1/f^2 and sqrt(4 - 3 f^2) (= sqrt(1 + 3 (1 - f^2)), the speeds' S)
// between them.  S, 1/S, 1/(S+1) and 1/D^2 (D = 5 + 2S) come from one
// reciprocal.
__device__ __forceinline__ void closure_and_prep(float N, float Fx, float Fy, float Fz,
                                                 float inv_c, double c_d, float ns, Press &P,
                                                 SpeedPrep &sp)
{
    sp = SpeedPrep{};
    sp.iso = true;
    if (!(N > N_TINY)) {
        P.xx = P.yy = P.zz = P.xy = P.xz = P.yz = 0.0f;
        return;
    }
    const float q = inv_c * frcp(N);
    sp.ux = Fx * q;
    sp.uy = Fy * q;
    sp.uz = Fz * q;
    sp.x2 = sp.ux * sp.ux;
    sp.y2 = sp.uy * sp.uy;
    sp.z2 = sp.uz * sp.uz;
    const float f2 = sp.x2 + sp.y2 + sp.z2;
    const float Ns = N * ns;
    float S = 2.0f;   // sqrt(4 - 3 f^2) at f^2 <= 1e-20
    float inv_f2 = 0.0f;
    if (f2 > 1e-20f) {
        sp.iso = false;
        const double cn = double(N) * c_d;
        const double diff = cn * cn - (double(Fx) * double(Fx) + double(Fy) * double(Fy) +
                                       double(Fz) * double(Fz));
        // 1 - f^2 = diff q^2, the product in FP64 (q^2 = 1/(cN)^2 leaves the
        // FP32 range for N just above N_TINY)
        const double qd = double(q);
        const float g2 = diff > 0.0 ? float(diff * (qd * qd)) : 0.0f;
        const float fs = 1.0f - g2;
        S = fsqrt(1.0f + 3.0f * g2);
        const float Sp1 = S + 1.0f;
        const float D = 5.0f + 2.0f * S;
        const float D2 = D * D;
        const float R = frcp(S * Sp1 * D2);
        const float inv_S = R * Sp1 * D2;
        const float inv_Sp1 = R * S * D2;
        const float inv_D2 = R * S * Sp1;
        sp.Sm1 = 3.0f * g2 * inv_Sp1;
        sp.Q = (8.0f * D + 6.0f * (3.0f + 4.0f * fs) * inv_S) * inv_D2;
        sp.pref = (8.0f / 3.0f) * sp.Sm1 * inv_S * inv_S;
        inv_f2 = frcp(f2);
        sp.inv_f2 = inv_f2;
    }
    // Levermore chi with f^2 clamped to 1 and the speeds' S in place of
    // sqrt(4 - 3 f^2)
    const float f2c = rmin(f2, 1.0f);
    const float chi = (3.0f + 4.0f * f2c) * frcp(5.0f + 2.0f * S);
    const float iso = 0.5f * (1.0f - chi) * Ns;
    // (the anisotropic part is of order f^2 N: nothing at f^2 <= 1e-20)
    const float w = sp.iso ? 0.0f : 0.5f * (3.0f * chi - 1.0f) * Ns * inv_f2;
    P.xx = iso + w * sp.x2;
    P.yy = iso + w * sp.y2;
    P.zz = iso + w * sp.z2;
    P.xy = w * sp.ux * sp.uy;
    P.xz = w * sp.ux * sp.uz;
    P.yz = w * sp.uy * sp.uz;
}

__device__ __forceinline__ Speeds m1_axes(const SpeedPrep &p)
{
    Speeds s;
    m1_axis(p, p.ux, p.x2, p.y2 + p.z2, s.xm, s.xp);
    m1_axis(p, p.uy, p.y2, p.x2 + p.z2, s.ym, s.yp);
    m1_axis(p, p.uz, p.z2, p.x2 + p.y2, s.zm, s.zp);
    return s;
}

// HLL face flux of one component with speeds (units of c) lm*, lp* on the
// two sides: a+ = c max(0, lpL, lpR), a- = c min(0, lmL, lmR),
// G = (a+ GL - a- GR + a+ a- (UR - UL)) / (a+ - a-).
struct HllW {
    float wl, wr, wd;   // G = wl GL + wr GR + wd (UR - UL)
};

__device__ __forceinline__ HllW hll_weights(float lmL, float lpL, float lmR, float lpR, float c)
{
    // (the factor c keeps a+ - a- out of the denormal range where both
    // speeds nearly vanish, across a free-streaming beam: its reciprocal
    // stays finite)
    const float ap = c * rmax(0.0f, rmax(lpL, lpR));
    const float am = c * rmin(0.0f, rmin(lmL, lmR));
    const float den = ap - am;
    if (!(den > 0.0f)) return HllW{0.5f, 0.5f, 0.0f};
    const float w = frcp(den);
    return HllW{ap * w, -am * w, ap * am * w};
}

// ------------------------------------------------------- hydrogen rates
// alpha_B and case-B recombination cooling: Hui & Gnedin (1997);
// collisional ionisation, its cooling (13.6 eV each), collisional excitation
// and free-free cooling: Cen (1992).  Cooling rates are returned divided by
// 3/2 kB so that the energy update works in kelvin.  rates_f32 serves the
// FP32 chemistry (hardware exp2/log2), rates_f64 the FP64 chemistry (libm
// double precision).
template <typename R>
struct RateSetT {
    R alpha;  // [cm^3/s]
    R beta;   // [cm^3/s]
    R crb;    // (recombination + free-free) cooling / (1.5 kB) [K cm^3/s]
    R cci;    // (excitation + ionisation) cooling / (1.5 kB) [K cm^3/s]
};
using RateSet = RateSetT<float>;

__device__ __forceinline__ RateSet rates_f32(float T, float inv15kB)
{
    RateSet r;
    const float iT = frcp(T);
    const float lg = flog2(315614.0f * iT);           // log2(lambda)
    const float log2T = 18.2678016762f - lg;
    r.alpha = 2.753e-14f *
              fexp2(1.5f * lg - 2.242f * flog2(1.0f + fexp2(0.407f * lg - 0.5918495885f)));
    const float recb = 3.435e-30f * T *
                       fexp2(1.970f * lg - 3.720f * flog2(1.0f + fexp2(0.376f * lg - 0.4398918005f)));
    const float sT = fsqrt(T);
    const float damp = frcp(1.0f + sT * 3.162277660168e-3f);
    r.beta = 5.85e-11f * sT * fexp2(-227670.405977f * iT) * damp;
    const float colex = 7.5e-19f * fexp2(-170740.072699f * iT) * damp;
    const float colion = 2.178960222240e-11f * r.beta;
    const float lt = 5.5f - 0.301029995664f * log2T;
    const float brems = 1.42e-27f * sT * (1.1f + 0.34f * fexp2(-0.480898346963f * lt * lt));
    r.crb = (recb + brems) * inv15kB;
    r.cci = (colex + colion) * inv15kB;
    return r;
}

__device__ __forceinline__ RateSetT<double> rates_f64(double T, double inv15kB)
{
    RateSetT<double> r;
    const double lam = 315614.0 / T;                  // 2 T_HI / T
    const double llam = log(lam);
    r.alpha = 2.753e-14 * exp(1.5 * llam - 2.242 * log1p(exp(0.407 * (llam - log(2.740)))));
    const double recb =
        3.435e-30 * T * exp(1.970 * llam - 3.720 * log1p(exp(0.376 * (llam - log(2.250)))));
    const double sT = sqrt(T);
    const double damp = 1.0 / (1.0 + sT * 3.1622776601683795e-3);
    r.beta = 5.85e-11 * sT * exp(-157809.1 / T) * damp;
    const double colex = 7.5e-19 * exp(-118348.0 / T) * damp;
    const double colion = 2.178960222240e-11 * r.beta;   // 13.6 eV per ionisation
    const double lt = 5.5 - log10(T);
    const double brems = 1.42e-27 * sT * (1.1 + 0.34 * exp(-lt * lt / 3.0));
    r.crb = (recb + brems) * inv15kB;
    r.cci = (colex + colion) * inv15kB;
    return r;
}

// ------------------------------------------------ per-cell operator Phi
template <typename R>
struct ChemK {
    R dt, hfix, csig, T_h, T_floor, sub_eps, inv15kB;
};

__device__ __forceinline__ RateSetT<float> rates_of(float T, const ChemK<float> &K)
{
    return rates_f32(T, K.inv15kB);
}
__device__ __forceinline__ RateSetT<double> rates_of(double T, const ChemK<double> &K)
{
    return rates_f64(T, K.inv15kB);
}

// Adaptive sub-cycle time scale: the shorter of xHI / (gross xHI rate) and
// u / (heating + cooling rate).  Gross rates keep it well conditioned near
// equilibrium, where the net rate is a small difference of large terms.
template <typename R>
__device__ __forceinline__ R chem_timescale(int chem, const ChemK<R> &K, const RateSetT<R> &rs,
                                            R cR, R cI, R nH, R N, R xHI, R x, R T)
{
    R g = cI * K.csig * N;
    R gx = cR * rs.alpha * nH * x * x + (g + rs.beta * nH * x) * xHI;
    R t = R(3.0e38f);
    if (gx > R(0)) t = xHI * frcp(gx);
    if (chem == RT_CHEM_FULL) {
        R gu = g * xHI * K.T_h + nH * (x * x * cR * rs.crb + x * xHI * rs.cci);
        if (gu > R(0)) t = rmin(t, (R(1) + x) * T * frcp(gu));
    }
    return t;
}

// Subgrid clumping factors (Sec. 3.2.1) of a cell: C_R = max(1, norm_R
// nH^exp_R) and C_I = norm_I nH^exp_I.  FP32: 2^(exp log2 nH + l2n) with
// l2n = log2 norm; FP64: libm pow.  Exactly 1 when clumping is off.
__device__ __forceinline__ void clump_f32(const ClumpLaw &L, float nH, float &cR, float &cI)
{
    cR = 1.0f;
    cI = 1.0f;
    if (L.on) {
        const float l = flog2(nH);
        cR = rmax(1.0f, fexp2(L.cr_exp * l + L.cr_l2n));
        cI = fexp2(L.ci_exp * l + L.ci_l2n);
    }
}

__device__ __forceinline__ void clump_f64(const ClumpLawD &L, double nH, double &cR, double &cI)
{
    cR = 1.0;
    cI = 1.0;
    if (L.on) {
        cR = fmax(1.0, L.cr_norm * pow(nH, L.cr_exp));
        cI = L.ci_norm * pow(nH, L.ci_exp);
    }
}

// One sub-cycle of length h with the rates rs at the sub-cycle's starting
// T: implicit photon-conserving photoionisation, creation/destruction
// recombination update, semi-implicit energy update.  cR multiplies the
// terms in ne nHII (recombination and its cooling, bremsstrahlung), cI the
// photoionisation rate.  The ionised fraction xi is carried beside xHI with
// updates free of cancellation: 1 - xHI would lose its relative precision
// in nearly neutral gas, where cooling goes as its square.  N, xHI, xi, T
// updated; `absorbed` gains the photon density removed.
template <typename R>
__device__ __forceinline__ void chem_sub(int chem, const ChemK<R> &K, const RateSetT<R> &rs,
                                         R cR, R cI, R nH, R inv_nH, R h, R &N, R &xHI,
                                         R &xi, R &T, R &absorbed)
{
    const R a = cI * K.csig * h;
    const R nHI = nH * xHI;
    if (chem == RT_CHEM_FROZEN) {
        R Nn = N * frcp(R(1) + a * nHI);
        absorbed += N - Nn;
        N = Nn;
        return;
    }
    // photoionisation: remaining photons Nn and neutrals un solve
    // a un Nn = N - Nn, un - Nn = nHI - N; each root taken in the
    // cancellation-free form for its sign of aD.  Without photons
    // nothing is absorbed and xHI is left exactly as it is.
    const R x0 = xi;
    R Pd = R(0), xh = xHI;
    if (N > R(0)) {
        const R aN = a * N, aH = a * nHI, aD = aH - aN;
        const R opd = R(1) + aD;
        const R s = fsqrt(opd * opd + R(4) * aN);
        R Nn, un;
        if (aD >= R(0)) {
            Nn = R(2) * N * frcp(opd + s);
            un = Nn + (nHI - N);
        } else {
            un = R(2) * nHI * frcp((R(1) - aD) + s);
            Nn = un - (nHI - N);
        }
        Nn = rmin(rmax(Nn, R(0)), N);
        un = rmin(rmax(un, R(0)), nHI);
        Pd = R(2) * aN * nHI * frcp(R(1) + aN + aH + s);
        absorbed += N - Nn;
        N = Nn;
        xh = un * inv_nH;
    }

    // recombination (case B) and collisional ionisation:
    // xn = (xh + A x^2) / (1 + B x); with xh + x = 1 the ionised
    // fraction after it is x (1 + B - A x) / (1 + B x), taken in that
    // form when it is the smaller of the two
    const R x = rmin(x0 + Pd * inv_nH, R(1));
    const R A = cR * rs.alpha * nH * h, B = rs.beta * nH * h;
    const R den = frcp(R(1) + B * x);
    R xn = (xh + A * x * x) * den;
    R xin;
    if (xn >= R(0.5)) {
        xin = rmax(x * (R(1) + B - A * x) * den, R(0));
        xn = R(1) - xin;
    } else {
        xin = R(1) - xn;
    }
    xn = rmin(rmax(xn, R(1e-12)), R(1));

    // internal energy 3/2 kB nH (1+x) T: photo-heating, then cooling
    if (chem == RT_CHEM_FULL) {
        const R x1 = xin;
        const R lu = h * nH * (x1 * x1 * cR * rs.crb + x1 * xn * rs.cci) *
                     frcp((R(1) + x0) * T);
        const R Tn = ((R(1) + x0) * T + Pd * inv_nH * K.T_h) *
                     frcp((R(1) + lu) * (R(1) + x1));
        T = rmax(Tn, K.T_floor);
    }
    xHI = xn;
    xi = rmin(xin, R(1));
}

// Sub-cycles of one cell: fixed (nsub of length dt / nsub) or adaptive
// (h = min(rest, sub_eps t_chem), at most nsub, the last taking the rest).
// Returns the number of sub-cycles; N, xHI, T updated; `absorbed` gains the
// photon density removed.
template <typename R>
__device__ __forceinline__ int chem_cell(int chem, int nsub, int adaptive, const ChemK<R> &K,
                                         R cR, R cI, R nH, R &N, R &xHI, R &T, R &absorbed)
{
    const R inv_nH = frcp(nH);
    R xi = R(1) - xHI;
    R remaining = K.dt;
    int it = 0;
    for (; it < nsub && remaining > R(0); ++it) {
        RateSetT<R> rs;
        bool have = false;
        R h;
        if (it == nsub - 1) {
            h = remaining;
        } else if (adaptive) {
            rs = rates_of(T, K);
            have = true;
            h = rmin(remaining,
                     K.sub_eps * chem_timescale<R>(chem, K, rs, cR, cI, nH, N, xHI, xi, T));
        } else {
            h = K.hfix;
        }
        remaining -= h;
        if (it == nsub - 1 || remaining < R(0)) remaining = R(0);
        if (!have) rs = rates_of(T, K);
        chem_sub<R>(chem, K, rs, cR, cI, nH, inv_nH, h, N, xHI, xi, T, absorbed);
    }
    return it;
}

__device__ __forceinline__ int hist_bin(int n)
{
    int b = 31 - __builtin_clz(n > 0 ? n : 1);
    return b > 7 ? 7 : b;
}

}  // namespace rtk

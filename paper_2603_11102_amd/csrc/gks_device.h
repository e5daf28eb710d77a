// gks_device.h -- device math of the high-order isothermal GKS step (gfx950).
//
// Reconstruction (Section 2: fifth-order WENO-JS, dimension by dimension, to the 2x2 Gauss points of
// each face) and the gas-kinetic flux of the interface distribution f = g0 (1 - tau (a.u + A) + A t)
// (Section 2, Eq. (flux); coefficients from the moment system of the Appendix).
//
// Cells have unit width in the stencil formulas; derivatives are scaled by 1/h by the caller.
// Gauss points of a cell are xi = s sqrt(3)/6, s = -1 (m = 0) and s = +1 (m = 1).
//
// Flux: for the isothermal Maxwellian g0 with macroscopic state Q0 and spatial derivatives dQ0/dx_k,
// the moments of f reduce exactly (the Chapman-Enskog identities of the BGK model) to
//   F0 = E_n(Q0) - mu (dU/dx_n + grad U_n)            (no viscous mass flux, no bulk term),
//   F1 = J_n(Q0) Qdot,  Qdot = -sum_k J_k(Q0) dQ0/dx_k  (rho0 <u_n A psi> with A from compatibility),
// where E_k is the isothermal Euler flux and J_k its Jacobian; tau p0 = mu. The constant reference
// pressure c^2 rho_ref is dropped from E_n: it is the same at every face and cancels in the divergence,
// which keeps the O(Ma^2) pressure differences in FP32.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace gks {

template <typename real> struct Rc;
template <> struct Rc<float> {
    static __device__ __forceinline__ float erf_(float x) { return erff(x); }
    static __device__ __forceinline__ float exp_(float x) { return expf(x); }
    static __device__ __forceinline__ float expm1_(float x) { return expm1f(x); }
};
template <> struct Rc<double> {
    static __device__ __forceinline__ double erf_(double x) { return erf(x); }
    static __device__ __forceinline__ double exp_(double x) { return exp(x); }
    static __device__ __forceinline__ double expm1_(double x) { return expm1(x); }
};

#define GKS_SQRT3 1.7320508075688772935274463415059

// Reciprocal: FP32 uses the hardware v_rcp_f32 (about 1 ulp); FP64 refines v_rcp_f64 by two Newton
// steps (about 1 ulp). Arguments are positive normal numbers here (densities, WENO denominators).
template <typename real> __device__ __forceinline__ real rcp(real x);
template <> __device__ __forceinline__ float rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ __forceinline__ double rcp<double>(double x) {
    double y = __builtin_amdgcn_rcp(x);
    y = fma(fma(-x, y, 1.0), y, y);
    y = fma(fma(-x, y, 1.0), y, y);
    return y;
}

// ---------------------------------------------------------------------------------------------
// WENO-JS on five cells q[-2..2], written in the stencil's first differences
// d1 = q[-1] - q[-2], d2 = q[0] - q[-1], d3 = q[1] - q[0], d4 = q[2] - q[1]. Sub-stencil k's quadratic
// (cells k-2..k) has second difference a_k and twice its slope at the cell centre b_k (unit cells):
//   a0 = d2 - d1, b0 = 3 d2 - d1;   a1 = d3 - d2, b1 = d2 + d3;   a2 = d4 - d3, b2 = 3 d3 - d4,
// so that its smoothness indicator is 4 beta_k = (13/3) a_k^2 + b_k^2, its values at the faces
// xi = +-1/2 are q0 + (a_k +- 3 b_k)/12 and at the Gauss points xi = s sqrt3/6 q0 + s (sqrt3/12) b_k
// (the two-point Gauss rule integrates the quadratic exactly, so its even part there is q0).
// P_k = prod_{j != k} (4 eps + 4 beta_j)^2: the nonlinear weights gamma_k / (eps + beta_k)^2,
// normalised, equal gamma_k P_k / sum_j gamma_j P_j (the common factor 4^4 cancels), so one reciprocal
// per evaluation point suffices.
// ---------------------------------------------------------------------------------------------
template <typename real>
__device__ __forceinline__ void js_parts(real qm2, real qm1, real q0, real qp1, real qp2, real eps,
                                         real a[3], real b[3], real P[3]) {
    const real d1 = qm1 - qm2, d2 = q0 - qm1, d3 = qp1 - q0, d4 = qp2 - qp1;
    a[0] = d2 - d1;
    b[0] = real(3) * d2 - d1;
    a[1] = d3 - d2;
    b[1] = d2 + d3;
    a[2] = d4 - d3;
    b[2] = real(3) * d3 - d4;
    const real c133 = real(13.0 / 3.0), e4 = real(4) * eps;
    real e[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        e[k] = e4 + c133 * a[k] * a[k] + b[k] * b[k];
        e[k] *= e[k];
    }
    P[0] = e[1] * e[2];
    P[1] = e[0] * e[2];
    P[2] = e[0] * e[1];
}

// Face values of cell 0: right face (xi = +1/2, linear weights 1/10, 3/5, 3/10) and left face
// (xi = -1/2, weights 3/10, 3/5, 1/10). Both share the cell's smoothness indicators. The weights are
// divided by 3/5, and the 1/12 of the sub-stencil values goes into the denominator.
template <typename real>
__device__ __forceinline__ void weno_faces(real qm2, real qm1, real q0, real qp1, real qp2, real eps,
                                           real& right, real& left) {
    real a[3], b[3], P[3];
    js_parts(qm2, qm1, q0, qp1, qp2, eps, a, b, P);
    const real P1x = real(12) * P[1];
    real X0 = P[0] * (a[0] + real(3) * b[0]);
    real X1 = P[1] * (a[1] + real(3) * b[1]);
    real X2 = P[2] * (a[2] + real(3) * b[2]);
    right = q0 + (real(1.0 / 6.0) * X0 + (real(0.5) * X2 + X1)) *
                     rcp<real>(real(2) * P[0] + (real(6) * P[2] + P1x));
    X0 = P[0] * (a[0] - real(3) * b[0]);
    X1 = P[1] * (a[1] - real(3) * b[1]);
    X2 = P[2] * (a[2] - real(3) * b[2]);
    left = q0 + (real(0.5) * X0 + (real(1.0 / 6.0) * X2 + X1)) *
                    rcp<real>(real(6) * P[0] + (real(2) * P[2] + P1x));
}

// Linear weights at the Gauss points s = +-1 that reproduce the quartic: (7/36 - s sqrt3/1080, 11/18,
// 7/36 + s sqrt3/1080), here divided by 11/18 (WGL: the s = +1 outer weight of sub-stencil 0, WGH the
// other one).
#define GKS_WGL ((7.0 / 36.0 - GKS_SQRT3 / 1080.0) / (11.0 / 18.0))
#define GKS_WGH ((7.0 / 36.0 + GKS_SQRT3 / 1080.0) / (11.0 / 18.0))

// WENO-JS values at the two Gauss points of cell 0, vm (s = -1) and vp (s = +1). The sqrt3/12 of the
// sub-stencil deviations goes into the denominators.
template <typename real>
__device__ __forceinline__ void weno_gauss(real qm2, real qm1, real q0, real qp1, real qp2, real eps,
                                           real& vm, real& vp) {
    real a[3], b[3], P[3];
    js_parts(qm2, qm1, q0, qp1, qp2, eps, a, b, P);
    const real lo = real(GKS_WGL), hi = real(GKS_WGH), k = real(12.0 / GKS_SQRT3);
    const real X0 = P[0] * b[0], X1 = P[1] * b[1], X2 = P[2] * b[2];
    const real P1k = k * P[1];
    vp = q0 + (lo * X0 + (hi * X2 + X1)) * rcp<real>(real(k * lo) * P[0] + (real(k * hi) * P[2] + P1k));
    vm = q0 - (hi * X0 + (lo * X2 + X1)) * rcp<real>(real(k * hi) * P[0] + (real(k * lo) * P[2] + P1k));
}

// Quartic through five cell averages: values at the two Gauss points.
// value = e.q + s sqrt3 o.q, e = (-1/4320, 1/1080, 719/720, 1/1080, -1/4320),
// o = (7/432, -25/216, 0, 25/216, -7/432).
template <typename real>
__device__ __forceinline__ void quartic_gauss_value(real qm2, real qm1, real q0, real qp1, real qp2,
                                                    real& vm, real& vp) {
    real ev = real(-1.0 / 4320.0) * (qm2 + qp2) + real(1.0 / 1080.0) * (qm1 + qp1) + real(719.0 / 720.0) * q0;
    real od = real(GKS_SQRT3) * (real(7.0 / 432.0) * (qm2 - qp2) + real(25.0 / 216.0) * (qp1 - qm1));
    vm = ev - od;
    vp = ev + od;
}

// Quartic through five cell averages: derivatives (per unit cell) at the two Gauss points.
// e = (1/12, -2/3, 0, 2/3, -1/12), o = (-1/54, 13/54, -4/9, 13/54, -1/54).
template <typename real>
__device__ __forceinline__ void quartic_gauss_deriv(real qm2, real qm1, real q0, real qp1, real qp2,
                                                    real& dm, real& dp) {
    real ev = real(1.0 / 12.0) * (qm2 - qp2) + real(2.0 / 3.0) * (qp1 - qm1);
    real od = real(GKS_SQRT3) * (real(-1.0 / 54.0) * (qm2 + qp2) + real(13.0 / 54.0) * (qm1 + qp1) -
                                 real(4.0 / 9.0) * q0);
    dm = ev - od;
    dp = ev + od;
}

// erf(a) - erf(b) without cancellation when a ~ b in FP32: three-point Gauss-Legendre quadrature of
// (2/sqrt(pi)) exp(-t^2) over [b, a] (relative error < 2e-8 for |a - b| < 1/4).
template <typename real>
__device__ __forceinline__ real erf_diff(real a, real b) {
    return Rc<real>::erf_(a) - Rc<real>::erf_(b);
}
template <>
__device__ __forceinline__ float erf_diff<float>(float a, float b) {
    float h = 0.5f * (a - b);
    if (fabsf(h) < 0.125f) {
        float m = 0.5f * (a + b);
        const float x1 = 0.77459666924148338f;  // sqrt(3/5)
        float t0 = m - h * x1, t2 = m + h * x1;
        float s = (5.0f / 9.0f) * (expf(-t0 * t0) + expf(-t2 * t2)) + (8.0f / 9.0f) * expf(-m * m);
        return 1.1283791670955126f * h * s;  // 2/sqrt(pi)
    }
    return erff(a) - erff(b);
}

// Kinetic-average transcendentals: erf(aL), erf(aR), erf(aL) - erf(aR) and expm1(x).
// FP64: library functions. FP32, when |aL|, |aR| <= 1/4: the Maclaurin series of erf through x^9,
// erf(x) = (2/sqrt(pi)) x P(x^2) with P(y) = 1 - y/3 + y^2/10 - y^3/42 + y^4/216 (truncation < 1e-9
// relative), and for the difference, with A = a^2, B = b^2,
//   erf(a) - erf(b) = (2/sqrt(pi)) (a - b) [P(A) + b (a + b) Q(A, B)],  P(A) - P(B) = (A - B) Q(A, B),
//   Q = -1/3 + (A + B)/10 - (A^2 + AB + B^2)/42 + (A + B)(A^2 + B^2)/216,
// which has no cancellation when a ~ b (truncation < 1e-8 relative); expm1 by its series through x^5
// when |x| <= 1/16.
template <typename real>
struct KinTrans {
    static __device__ __forceinline__ void erfs(real aL, real aR, real& eL, real& eR, real& ed) {
        eL = Rc<real>::erf_(aL);
        eR = Rc<real>::erf_(aR);
        ed = erf_diff<real>(aL, aR);
    }
    static __device__ __forceinline__ real expm1_(real x) { return Rc<real>::expm1_(x); }
};
template <>
struct KinTrans<float> {
    static __device__ __forceinline__ float poly(float y) {
        float p = fmaf(y, 1.0f / 216.0f, -1.0f / 42.0f);
        p = fmaf(y, p, 0.1f);
        p = fmaf(y, p, -1.0f / 3.0f);
        return fmaf(y, p, 1.0f);
    }
    static __device__ __forceinline__ void erfs(float aL, float aR, float& eL, float& eR, float& ed) {
        const float k2 = 1.1283791670955126f;  // 2/sqrt(pi)
        if (fabsf(aL) <= 0.25f && fabsf(aR) <= 0.25f) {
            const float A = aL * aL, B = aR * aR;
            const float PA = poly(A);
            eL = k2 * aL * PA;
            eR = k2 * aR * poly(B);
            const float sAB = A + B, pAB = A * B;
            const float u = fmaf(sAB, sAB, -pAB);  // A^2 + AB + B^2
            const float Q = fmaf(sAB * (u - pAB), 1.0f / 216.0f, fmaf(u, -1.0f / 42.0f, fmaf(sAB, 0.1f, -1.0f / 3.0f)));
            ed = k2 * (aL - aR) * fmaf(aR * (aL + aR), Q, PA);
        } else {
            eL = erff(aL);
            eR = erff(aR);
            ed = erf_diff<float>(aL, aR);
        }
    }
    static __device__ __forceinline__ float expm1_(float x) {
        if (fabsf(x) <= 0.0625f) {
            float p = fmaf(x, 1.0f / 120.0f, 1.0f / 24.0f);
            p = fmaf(x, p, 1.0f / 6.0f);
            p = fmaf(x, p, 0.5f);
            p = fmaf(x, p, 1.0f);
            return x * p;
        }
        return expm1f(x);
    }
};

// FP64, when |aL|, |aR| <= 1/4: the Maclaurin series of erf through x^21 (truncation < 1e-22
// relative), the difference from the same S_k recurrence, and expm1 through x^11 when |x| <= 1/16;
// otherwise the library functions.
template <>
struct KinTrans<double> {
    static __device__ __forceinline__ double series(double x2) {  // sum_k (-1)^k x2^k / (k! (2k+1))
        double p = 1.0 / 76204800.0;
        p = fma(x2, p, -1.0 / 6894720.0);
        p = fma(x2, p, 1.0 / 685440.0);
        p = fma(x2, p, -1.0 / 75600.0);
        p = fma(x2, p, 1.0 / 9360.0);
        p = fma(x2, p, -1.0 / 1320.0);
        p = fma(x2, p, 1.0 / 216.0);
        p = fma(x2, p, -1.0 / 42.0);
        p = fma(x2, p, 0.1);
        p = fma(x2, p, -1.0 / 3.0);
        return fma(x2, p, 1.0);
    }
    static __device__ __forceinline__ void erfs(double aL, double aR, double& eL, double& eR, double& ed) {
        const double k2 = 1.1283791670955125739;  // 2/sqrt(pi)
        if (fabs(aL) <= 0.25 && fabs(aR) <= 0.25) {
            eL = k2 * aL * series(aL * aL);
            eR = k2 * aR * series(aR * aR);
            // (erf a - erf b) = (2/sqrt(pi)) (a - b) sum_k c_k S_{2k+1}, S_n = (a^n - b^n) / (a - b)
            const double p = aL + aR, q = aL * aR;
            const double c[11] = {1.0, -1.0 / 3.0, 0.1, -1.0 / 42.0, 1.0 / 216.0, -1.0 / 1320.0, 1.0 / 9360.0,
                                  -1.0 / 75600.0, 1.0 / 685440.0, -1.0 / 6894720.0, 1.0 / 76204800.0};
            double sm2 = 1.0, sm1 = p;  // S_1, S_2
            double acc = c[0];
#pragma unroll
            for (int k = 1; k <= 10; ++k) {
                const double s_odd = fma(p, sm1, -q * sm2);   // S_{2k+1}
                const double s_even = fma(p, s_odd, -q * sm1); // S_{2k+2}
                acc = fma(c[k], s_odd, acc);
                sm2 = s_odd;
                sm1 = s_even;
            }
            ed = k2 * (aL - aR) * acc;
        } else {
            eL = erf(aL);
            eR = erf(aR);
            ed = erf_diff<double>(aL, aR);
        }
    }
    static __device__ __forceinline__ double expm1_(double x) {
        if (fabs(x) <= 0.0625) {
            double p = 1.0 / 39916800.0;
            p = fma(x, p, 1.0 / 3628800.0);
            p = fma(x, p, 1.0 / 362880.0);
            p = fma(x, p, 1.0 / 40320.0);
            p = fma(x, p, 1.0 / 5040.0);
            p = fma(x, p, 1.0 / 720.0);
            p = fma(x, p, 1.0 / 120.0);
            p = fma(x, p, 1.0 / 24.0);
            p = fma(x, p, 1.0 / 6.0);
            p = fma(x, p, 0.5);
            p = fma(x, p, 1.0);
            return x * p;
        }
        return expm1(x);
    }
};

template <typename real>
struct FluxConst {
    real lam;      // lambda = Ma^2 / (2 U_ref^2)
    real sl;       // sqrt(lambda)
    real kk;       // 1 / (2 sqrt(pi lambda))
    real c2;       // 1 / (2 lambda)
    real mu;       // viscosity
    real rho_ref;  // reference density
};

// Gas-kinetic flux at one Gauss point, in the face's local frame: variables (rho', m_n, m_t1, m_t2),
// derivative directions (n, t1, t2). qL, qR: reconstructed left/right states; g[d][v]: dQ_v/dx_d.
// Adds w * F0 (if NEED_F0) and w * F1 to f0, f1.
// SHIFT: qL[1], qR[1] hold m_n - cm for a constant cm, and the mass-flux part of f0 receives F0 - cm
// (the constant cancels in the flux difference of a cell). The half-space weights satisfy
// hL + hR - 1 = (erf(aL) - erf(aR)) / 2, so the shifted mass flux carries no O(cm) rounding.
template <typename real, bool NEED_F0, bool SHIFT = false>
__device__ __forceinline__ void gp_flux(const real qL[4], const real qR[4], const real g[3][4],
                                        const FluxConst<real>& k, real w, real f0[4], real f1[4],
                                        real cm = real(0)) {
    // kinetic (half-space) average of the left and right Maxwellians, in deviation form
    real rL = k.rho_ref + qL[0], rR = k.rho_ref + qR[0];
    const real mL = SHIFT ? cm + qL[1] : qL[1], mR = SHIFT ? cm + qR[1] : qR[1];
    real uL = mL * rcp<real>(rL), uR = mR * rcp<real>(rR);
    real aL = k.sl * uL, aR = k.sl * uR;
    real eaL, eaR, ead;
    KinTrans<real>::erfs(aL, aR, eaL, eaR, ead);
    real hL = real(0.5) * (real(1) + eaL);
    real hR = real(0.5) * (real(1) - eaR);
    real eR = Rc<real>::exp_(-k.lam * uR * uR);
    real dE = eR * KinTrans<real>::expm1_(k.lam * (uR - uL) * (uR + uL));  // eL - eR
    real eL = eR + dE;                                                     // exp(-lambda uL^2)
    real rho0p = qL[0] * hL + qR[0] * hR + k.rho_ref * real(0.5) * ead;
    real m0[3];
    real mass_flux;  // F0 of the density: m0[0], or m0[0] - cm when shifted
    if (SHIFT) {
        mass_flux = qL[1] * hL + qR[1] * hR + real(0.5) * cm * ead +
                    k.kk * (qL[0] * eL - qR[0] * eR + k.rho_ref * dE);
        m0[0] = cm + mass_flux;
    } else {
        m0[0] = qL[1] * hL + qR[1] * hR + k.kk * (qL[0] * eL - qR[0] * eR + k.rho_ref * dE);
        mass_flux = m0[0];
    }
    m0[1] = qL[2] * hL + qR[2] * hR;
    m0[2] = qL[3] * hL + qR[3] * hR;
    real r0 = k.rho_ref + rho0p;
    real ir = rcp<real>(r0);
    real U[3] = {m0[0] * ir, m0[1] * ir, m0[2] * ir};
    if (NEED_F0) {
        // the velocity gradients dU[d][j] = (dm_j/dx_d - U_j drho/dx_d) / rho0 that the stress needs
        const real u00 = (g[0][1] - U[0] * g[0][0]) * ir;
        const real u01 = (g[0][2] - U[1] * g[0][0]) * ir, u10 = (g[1][1] - U[0] * g[1][0]) * ir;
        const real u02 = (g[0][3] - U[2] * g[0][0]) * ir, u20 = (g[2][1] - U[0] * g[2][0]) * ir;
        f0[0] += w * mass_flux;
        f0[1] += w * (m0[0] * U[0] + k.c2 * rho0p - k.mu * real(2) * u00);
        f0[2] += w * (m0[0] * U[1] - k.mu * (u01 + u10));
        f0[3] += w * (m0[0] * U[2] - k.mu * (u02 + u20));
    }
    // Euler time derivative of Q0. Its advection term needs no velocity gradient:
    // rho0 (U . grad) U_j = sum_d U_d dm_j/dx_d - U_j sum_d U_d drho/dx_d.
    real divm = g[0][1] + g[1][2] + g[2][3];
    real qd0 = -divm;
    const real H = (U[0] * g[0][0] + U[1] * g[1][0] + U[2] * g[2][0]) - divm;
    real qd[3];
#pragma unroll
    for (int j = 0; j < 3; ++j)
        qd[j] = U[j] * H - (U[0] * g[0][1 + j] + U[1] * g[1][1 + j] + U[2] * g[2][1 + j]) - k.c2 * g[j][0];
    f1[0] += w * qd[0];
    f1[1] += w * (real(2) * U[0] * qd[0] - U[0] * U[0] * qd0 + k.c2 * qd0);
    f1[2] += w * (U[1] * qd[0] + U[0] * qd[1] - U[0] * U[1] * qd0);
    f1[3] += w * (U[2] * qd[0] + U[0] * qd[2] - U[0] * U[2] * qd0);
}

// ---------------------------------------------------------------------------------------------
// Adjoint support (FP64): WENO evaluations that also return their normalised nonlinear weights, the
// sub-stencil coefficients those weights combine, and the reverse of gp_flux.
// ---------------------------------------------------------------------------------------------
template <typename real>
__device__ __forceinline__ void weno_faces_w(real qm2, real qm1, real q0, real qp1, real qp2, real eps,
                                             real& right, real& left, real wr[3], real wl[3]) {
    real a[3], b[3], P[3];
    js_parts(qm2, qm1, q0, qp1, qp2, eps, a, b, P);
    // weights divided by 3/5 and multiplied by 12 in the denominator, as in weno_faces
    const real P1x = real(12) * P[1];
    real c0 = real(2) * P[0], c2 = real(6) * P[2];
    real is = rcp<real>(c0 + (c2 + P1x));
    wr[0] = c0 * is;
    wr[1] = P1x * is;
    wr[2] = c2 * is;
    right = q0 + (real(1.0 / 6.0) * P[0] * (a[0] + real(3) * b[0]) +
                  (real(0.5) * P[2] * (a[2] + real(3) * b[2]) + P[1] * (a[1] + real(3) * b[1]))) * is;
    c0 = real(6) * P[0];
    c2 = real(2) * P[2];
    is = rcp<real>(c0 + (c2 + P1x));
    wl[0] = c0 * is;
    wl[1] = P1x * is;
    wl[2] = c2 * is;
    left = q0 + (real(0.5) * P[0] * (a[0] - real(3) * b[0]) +
                 (real(1.0 / 6.0) * P[2] * (a[2] - real(3) * b[2]) + P[1] * (a[1] - real(3) * b[1]))) * is;
}

template <typename real>
__device__ __forceinline__ void weno_gauss_w(real qm2, real qm1, real q0, real qp1, real qp2, real eps,
                                             real& vm, real& vp, real wm[3], real wp[3]) {
    real a[3], b[3], P[3];
    js_parts(qm2, qm1, q0, qp1, qp2, eps, a, b, P);
    const real lo = real(GKS_WGL), hi = real(GKS_WGH), r12 = real(GKS_SQRT3 / 12.0);
    const real X0 = P[0] * b[0], X1 = P[1] * b[1], X2 = P[2] * b[2];
    real c0 = lo * P[0], c2 = hi * P[2];
    real is = rcp<real>(c0 + (c2 + P[1]));
    wp[0] = c0 * is;
    wp[1] = P[1] * is;
    wp[2] = c2 * is;
    vp = q0 + r12 * (lo * X0 + (hi * X2 + X1)) * is;
    c0 = hi * P[0];
    c2 = lo * P[2];
    is = rcp<real>(c0 + (c2 + P[1]));
    wm[0] = c0 * is;
    wm[1] = P[1] * is;
    wm[2] = c2 * is;
    vm = q0 - r12 * (hi * X0 + (lo * X2 + X1)) * is;
}

// Coefficient of cell r (0..4 over the stencil -2..2) in sub-stencil k's value:
//   face xi = +1/2 (side 0) and xi = -1/2 (side 1); Gauss point s = -1 (side 2) and s = +1 (side 3).
__device__ __forceinline__ double sub_coef(int side, int k, int r) {
    const int l = r - k;
    if (l < 0 || l > 2) return 0.0;
    const double t = GKS_SQRT3;
    switch (side) {
        case 0: {
            const double c[3][3] = {{2.0 / 6, -7.0 / 6, 11.0 / 6}, {-1.0 / 6, 5.0 / 6, 2.0 / 6}, {2.0 / 6, 5.0 / 6, -1.0 / 6}};
            return c[k][l];
        }
        case 1: {
            const double c[3][3] = {{-1.0 / 6, 5.0 / 6, 2.0 / 6}, {2.0 / 6, 5.0 / 6, -1.0 / 6}, {11.0 / 6, -7.0 / 6, 2.0 / 6}};
            return c[k][l];
        }
        default: {
            const double s = side == 2 ? -1.0 : 1.0;
            const double c[3][3] = {{s * t / 12, -s * t / 3, 1.0 + s * t / 4},
                                    {-s * t / 12, 1.0, s * t / 12},
                                    {1.0 - s * t / 4, s * t / 3, -s * t / 12}};
            return c[k][l];
        }
    }
}

// Effective linear weight of stencil cell r for nonlinear weights w[3] on a given side.
__device__ __forceinline__ double weno_eff(int side, const double w[3], int r) {
    return w[0] * sub_coef(side, 0, r) + w[1] * sub_coef(side, 1, r) + w[2] * sub_coef(side, 2, r);
}

// Jacobian row dv/dq_r (r = 0..4 over the stencil -2..2) of a WENO-JS evaluation on `side` (as in
// sub_coef) with the nonlinear weights differentiated too. With e_k = 4 (eps + beta_k) the normalised
// weights are omega_k = (gamma_k / e_k^2) / sum_j (gamma_j / e_j^2), so
//   dv/dq_r = sum_k omega_k c_k[r] - 2 sum_k omega_k (v_k - v) (de_k/dq_r) / e_k,
// v_k the sub-stencil values and c_k[r] their coefficients. w: the weights, v: the value.
__device__ __forceinline__ void weno_jacobian(int side, const double q[5], double eps, const double w[3], double v,
                                              double J[5]) {
    const double c133 = 13.0 / 3.0, e4 = 4.0 * eps;
    // 4 beta_k = (13/3) a_k^2 + b_k^2 with a_k, b_k linear in the sub-stencil's cells
    const double a0 = q[0] - 2.0 * q[1] + q[2], b0 = q[0] - 4.0 * q[1] + 3.0 * q[2];
    const double a1 = q[1] - 2.0 * q[2] + q[3], b1 = q[1] - q[3];
    const double a2 = q[2] - 2.0 * q[3] + q[4], b2 = 3.0 * q[2] - 4.0 * q[3] + q[4];
    const double e[3] = {e4 + c133 * a0 * a0 + b0 * b0, e4 + c133 * a1 * a1 + b1 * b1, e4 + c133 * a2 * a2 + b2 * b2};
    double g[3];
    for (int k = 0; k < 3; ++k) {
        double vk = 0.0;
        for (int l = 0; l < 3; ++l) vk += sub_coef(side, k, k + l) * q[k + l];
        g[k] = -2.0 * w[k] * (vk - v) / e[k];
    }
    // de_k/dq over the sub-stencil's three cells: (26/3) a (1, -2, 1) + 2 b (db/dq)
    const double t0 = 26.0 / 3.0 * a0, t1 = 26.0 / 3.0 * a1, t2 = 26.0 / 3.0 * a2;
    const double d0[3] = {t0 + 2.0 * b0, -2.0 * t0 - 8.0 * b0, t0 + 6.0 * b0};
    const double d1[3] = {t1 + 2.0 * b1, -2.0 * t1, t1 - 2.0 * b1};
    const double d2[3] = {t2 + 6.0 * b2, -2.0 * t2 - 8.0 * b2, t2 + 2.0 * b2};
    for (int r = 0; r < 5; ++r) J[r] = weno_eff(side, w, r);
    for (int l = 0; l < 3; ++l) {
        J[l] += g[0] * d0[l];
        J[1 + l] += g[1] * d1[l];
        J[2 + l] += g[2] * d2[l];
    }
}

// Quartic Gauss value (deriv = 0) or derivative (deriv = 1) coefficient of stencil cell r at s.
__device__ __forceinline__ double quartic_coef(int deriv, int s, int r) {
    const double t = GKS_SQRT3;
    if (deriv == 0) {
        const double e[5] = {-1.0 / 4320, 1.0 / 1080, 719.0 / 720, 1.0 / 1080, -1.0 / 4320};
        const double o[5] = {7.0 / 432, -25.0 / 216, 0.0, 25.0 / 216, -7.0 / 432};
        return e[r] + s * t * o[r];
    }
    const double e[5] = {1.0 / 12, -2.0 / 3, 0.0, 2.0 / 3, -1.0 / 12};
    const double o[5] = {-1.0 / 54, 13.0 / 54, -4.0 / 9, 13.0 / 54, -1.0 / 54};
    return e[r] + s * t * o[r];
}

// Reverse of gp_flux (FP64): given the adjoints b0 (of the accumulated F0 contribution, stage 1
// only) and b1 (of F1), add the adjoints of the Gauss-point inputs to qLb, qRb, gb.
template <bool NEED_F0>
__device__ __forceinline__ void gp_flux_adj(const double qL[4], const double qR[4], const double g[3][4],
                                            const FluxConst<double>& k, double w, const double b0[4],
                                            const double b1[4], double qLb[4], double qRb[4], double gb[3][4]) {
    // ---- forward recompute
    const double rL = k.rho_ref + qL[0], rR = k.rho_ref + qR[0];
    const double irL = rcp<double>(rL), irR = rcp<double>(rR);
    const double uL = qL[1] * irL, uR = qR[1] * irR;
    const double aL = k.sl * uL, aR = k.sl * uR;
    // the forward's evaluation of erf(aL), erf(aR), erf(aL) - erf(aR) and expm1
    double EaL, EaR, Ead;
    KinTrans<double>::erfs(aL, aR, EaL, EaR, Ead);
    const double hL = 0.5 * (1.0 + EaL), hR = 0.5 * (1.0 - EaR);
    const double eR = exp(-k.lam * uR * uR), eL = exp(-k.lam * uL * uL);
    const double dE = eR * KinTrans<double>::expm1_(k.lam * (uR - uL) * (uR + uL));
    const double rho0p = qL[0] * hL + qR[0] * hR + k.rho_ref * 0.5 * Ead;
    double m0[3];
    m0[0] = qL[1] * hL + qR[1] * hR + k.kk * (qL[0] * eL - qR[0] * eR + k.rho_ref * dE);
    m0[1] = qL[2] * hL + qR[2] * hR;
    m0[2] = qL[3] * hL + qR[3] * hR;
    const double r0 = k.rho_ref + rho0p;
    const double ir = rcp<double>(r0);
    double U[3] = {m0[0] * ir, m0[1] * ir, m0[2] * ir};
    double dU[3][3];
    for (int d = 0; d < 3; ++d)
        for (int j = 0; j < 3; ++j) dU[d][j] = (g[d][1 + j] - U[j] * g[d][0]) * ir;
    const double divm = g[0][1] + g[1][2] + g[2][3];
    const double qd0 = -divm;
    double adv[3], qd[3];
    for (int j = 0; j < 3; ++j) {
        adv[j] = U[0] * dU[0][j] + U[1] * dU[1][j] + U[2] * dU[2][j];
        qd[j] = -U[j] * divm - r0 * adv[j] - k.c2 * g[j][0];
    }
    // ---- reverse
    double A1[4], A0[4];
    for (int v = 0; v < 4; ++v) {
        A1[v] = w * b1[v];
        A0[v] = NEED_F0 ? w * b0[v] : 0.0;
    }
    double Ub[3] = {0, 0, 0}, m0b[3] = {0, 0, 0}, dUb[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    double qdb[3] = {0, 0, 0};
    double qd0b = 0.0, r0b = 0.0, r0pb = 0.0, irb = 0.0, divmb = 0.0;
    // F1
    qdb[0] += A1[0];
    Ub[0] += A1[1] * (2.0 * qd[0] - 2.0 * U[0] * qd0);
    qdb[0] += A1[1] * 2.0 * U[0];
    qd0b += A1[1] * (-U[0] * U[0] + k.c2);
    for (int j = 1; j < 3; ++j) {
        Ub[j] += A1[1 + j] * (qd[0] - U[0] * qd0);
        Ub[0] += A1[1 + j] * (qd[j] - U[j] * qd0);
        qdb[0] += A1[1 + j] * U[j];
        qdb[j] += A1[1 + j] * U[0];
        qd0b += -A1[1 + j] * U[0] * U[j];
    }
    double advb[3];
    for (int j = 0; j < 3; ++j) {
        Ub[j] += -qdb[j] * divm;
        divmb += -qdb[j] * U[j];
        r0b += -qdb[j] * adv[j];
        advb[j] = -qdb[j] * r0;
        gb[j][0] += -k.c2 * qdb[j];
    }
    for (int j = 0; j < 3; ++j)
        for (int d = 0; d < 3; ++d) {
            Ub[d] += advb[j] * dU[d][j];
            dUb[d][j] += advb[j] * U[d];
        }
    divmb += -qd0b;
    gb[0][1] += divmb;
    gb[1][2] += divmb;
    gb[2][3] += divmb;
    // F0
    if (NEED_F0) {
        m0b[0] += A0[0];
        m0b[0] += A0[1] * U[0];
        Ub[0] += A0[1] * m0[0];
        r0pb += A0[1] * k.c2;
        dUb[0][0] += -2.0 * k.mu * A0[1];
        for (int j = 1; j < 3; ++j) {
            m0b[0] += A0[1 + j] * U[j];
            Ub[j] += A0[1 + j] * m0[0];
            dUb[0][j] += -k.mu * A0[1 + j];
            dUb[j][0] += -k.mu * A0[1 + j];
        }
    }
    // velocity gradients
    for (int d = 0; d < 3; ++d)
        for (int j = 0; j < 3; ++j) {
            gb[d][1 + j] += dUb[d][j] * ir;
            Ub[j] += -dUb[d][j] * g[d][0] * ir;
            gb[d][0] += -dUb[d][j] * U[j] * ir;
            irb += dUb[d][j] * dU[d][j] * r0;
        }
    for (int j = 0; j < 3; ++j) {
        m0b[j] += Ub[j] * ir;
        irb += Ub[j] * m0[j];
    }
    r0b += -irb * ir * ir;
    r0pb += r0b;
    // kinetic average
    double hLb = 0.0, hRb = 0.0, eLb = 0.0, eRb = 0.0, EaLb = 0.0, EaRb = 0.0;
    for (int j = 1; j < 3; ++j) {
        qLb[1 + j] += m0b[j] * hL;
        qRb[1 + j] += m0b[j] * hR;
        hLb += m0b[j] * qL[1 + j];
        hRb += m0b[j] * qR[1 + j];
    }
    qLb[1] += m0b[0] * hL;
    qRb[1] += m0b[0] * hR;
    hLb += m0b[0] * qL[1];
    hRb += m0b[0] * qR[1];
    qLb[0] += m0b[0] * k.kk * eL;
    qRb[0] += -m0b[0] * k.kk * eR;
    eLb += m0b[0] * k.kk * (qL[0] + k.rho_ref);
    eRb += -m0b[0] * k.kk * (qR[0] + k.rho_ref);
    qLb[0] += r0pb * hL;
    qRb[0] += r0pb * hR;
    hLb += r0pb * qL[0];
    hRb += r0pb * qR[0];
    EaLb += 0.5 * k.rho_ref * r0pb;
    EaRb += -0.5 * k.rho_ref * r0pb;
    EaLb += 0.5 * hLb;
    EaRb += -0.5 * hRb;
    const double c2pi = 1.1283791670955126;  // 2 / sqrt(pi)
    // d erf(sl u)/du = sl (2/sqrt(pi)) exp(-sl^2 u^2), and sl^2 = lambda: exp(-aL^2) is eL
    double uLb = k.sl * EaLb * c2pi * eL + eLb * eL * (-2.0 * k.lam * uL);
    double uRb = k.sl * EaRb * c2pi * eR + eRb * eR * (-2.0 * k.lam * uR);
    qLb[1] += uLb * irL;
    qLb[0] += -uLb * qL[1] * irL * irL;
    qRb[1] += uRb * irR;
    qRb[0] += -uRb * qR[1] * irR * irR;
}

}  // namespace gks

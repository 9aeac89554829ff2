// Device math for the AutoDiffGeo map: sigma_k (Tab. nonlinearfunctions),
// Rect1D and the in-plane factors of the primitives of Tab. autodiffgeo.
// Geometry is FP64; results are rounded to FP32 once, at the store.
#pragma once

#include "sg_internal.h"

namespace sg {

constexpr double kPiHalf = 1.5707963267948966;
constexpr double kInvSqrt2 = 0.70710678118654752;
constexpr double kInvSqrtPi = 0.56418958354775629;
// sigmoid / erf are taken as exactly 0 or 1 beyond these |t| (tails below
// 3.8e-11 and 2e-17); the support boxes use the same bounds, so results do not
// depend on how the grid is tiled.
constexpr double kSigmoidCut = 24.0;
constexpr double kErfCut = 6.0;

__host__ __device__ inline double sigma_cut(int kind) {
    switch (kind) {
        case SG_SIGMA_SIGMOID: return kSigmoidCut;
        case SG_SIGMA_ERF: return kErfCut;
        case SG_SIGMA_SIN: return kPiHalf;
        case SG_SIGMA_LINEAR: return 0.5;
        default: return kInvSqrt2;
    }
}

// Compile-time feature sets: which primitive types and which in-plane sigma
// kinds a kernel instantiation handles.  Scenes are dispatched to the smallest
// instantiation that covers them, so the common kernels carry no code for
// primitives or transcendental functions they never see.
enum : int { T_BOX = 1, T_ELL = 2, T_POLY = 4, T_GCART = 8, T_POLAR = 16, T_SERIES = 32, T_ALL = 63 };
enum : int { S_SIGMOID = 1, S_ERF = 2, S_SIN = 4, S_LIN = 8, S_QUAD = 16, S_ALL = 31 };

// ---- one function per kind: value, and value + d/dt

// Logistic sigmoid for |t| < kSigmoidCut in FP64.  With a = |t|,
// e^-a = 2^n e^x where n = rint(-a log2 e) and |x| <= ln(2) / 2; e^x is the
// degree-9 Taylor polynomial (truncation below 1e-11 relative), 2^n an exponent
// shift, and 1 / (1 + e^-a) takes the hardware reciprocal plus two Newton steps.
// sigma(t) = 1 / (1 + e^-a) for t >= 0 and e^-a / (1 + e^-a) for t < 0.
__device__ __forceinline__ double sigm_core(double t) {
    constexpr double kLog2e = 1.4426950408889634;
    constexpr double kLn2 = 0.69314718055994531;
    const double a = fabs(t);
    const double y = -a * kLog2e;
    const double n = rint(y);
    const double x = (y - n) * kLn2;
    double p = 1.0 / 362880.0;
    p = fma(p, x, 1.0 / 40320.0);
    p = fma(p, x, 1.0 / 5040.0);
    p = fma(p, x, 1.0 / 720.0);
    p = fma(p, x, 1.0 / 120.0);
    p = fma(p, x, 1.0 / 24.0);
    p = fma(p, x, 1.0 / 6.0);
    p = fma(p, x, 0.5);
    p = fma(p, x, 1.0);
    p = fma(p, x, 1.0);
    const double e = ldexp(p, (int)n);          // e^-a in (0, 1]
    const double d = 1.0 + e;                   // in (1, 2]
    double r = __builtin_amdgcn_rcp(d);
    r = fma(r, fma(-d, r, 1.0), r);
    r = fma(r, fma(-d, r, 1.0), r);
    return t >= 0.0 ? r : e * r;
}
__device__ __forceinline__ double sigm_v(double t) {
    if (t <= -kSigmoidCut) return 0.0;
    if (t >= kSigmoidCut) return 1.0;
    return sigm_core(t);
}
__device__ __forceinline__ void sigm_vd(double t, double& s, double& ds) {
    if (t <= -kSigmoidCut) { s = 0.0; ds = 0.0; return; }
    if (t >= kSigmoidCut) { s = 1.0; ds = 0.0; return; }
    s = sigm_core(t);
    ds = s * (1.0 - s);
}
__device__ __forceinline__ double erf_v(double t) {
    if (t <= -kErfCut) return 0.0;
    if (t >= kErfCut) return 1.0;
    return 0.5 * (1.0 + erf(t));
}
__device__ __forceinline__ void erf_vd(double t, double& s, double& ds) {
    if (t <= -kErfCut) { s = 0.0; ds = 0.0; return; }
    if (t >= kErfCut) { s = 1.0; ds = 0.0; return; }
    s = 0.5 * (1.0 + erf(t));
    ds = exp(-t * t) * kInvSqrtPi;
}
__device__ __forceinline__ double sin_v(double t) {
    if (t < -kPiHalf) return 0.0;
    if (t > kPiHalf) return 1.0;
    return 0.5 * (1.0 + sin(t));
}
__device__ __forceinline__ void sin_vd(double t, double& s, double& ds) {
    if (t < -kPiHalf) { s = 0.0; ds = 0.0; return; }
    if (t > kPiHalf) { s = 1.0; ds = 0.0; return; }
    double sn, cs;
    sincos(t, &sn, &cs);
    s = 0.5 * (1.0 + sn);
    ds = (t > -kPiHalf && t < kPiHalf) ? 0.5 * cs : 0.0;
}
__device__ __forceinline__ double lin_v(double t) { return fmax(0.0, fmin(1.0, t + 0.5)); }
__device__ __forceinline__ void lin_vd(double t, double& s, double& ds) {
    s = fmax(0.0, fmin(1.0, t + 0.5));
    ds = (t > -0.5 && t < 0.5) ? 1.0 : 0.0;
}
__device__ __forceinline__ double quad_v(double t) {
    if (t < -kInvSqrt2) return 0.0;
    if (t < 0.0) { const double a = kInvSqrt2 + t; return a * a; }
    if (t <= kInvSqrt2) { const double a = kInvSqrt2 - t; return 1.0 - a * a; }
    return 1.0;
}
__device__ __forceinline__ void quad_vd(double t, double& s, double& ds) {
    if (t < -kInvSqrt2) { s = 0.0; ds = 0.0; return; }
    if (t < 0.0) { const double a = kInvSqrt2 + t; s = a * a; ds = 2.0 * a; return; }
    if (t <= kInvSqrt2) {
        const double a = kInvSqrt2 - t;
        s = 1.0 - a * a;
        ds = (t < kInvSqrt2) ? 2.0 * a : 0.0;
        return;
    }
    s = 1.0;
    ds = 0.0;
}
// out-of-line copies of the transcendental kinds for the catch-all kernels
// (value and derivative come back as one pair, in registers)
static __device__ __noinline__ double sigm_v_call(double t) { return sigm_v(t); }
static __device__ __noinline__ double2 sigm_vd_call(double t) {
    double s, ds;
    sigm_vd(t, s, ds);
    return make_double2(s, ds);
}
static __device__ __noinline__ double erf_v_call(double t) { return erf_v(t); }
static __device__ __noinline__ double2 erf_vd_call(double t) {
    double s, ds;
    erf_vd(t, s, ds);
    return make_double2(s, ds);
}
static __device__ __noinline__ double sin_v_call(double t) { return sin_v(t); }
static __device__ __noinline__ double2 sin_vd_call(double t) {
    double s, ds;
    sin_vd(t, s, ds);
    return make_double2(s, ds);
}

// sigma(t) for a kind drawn from SIGS
template <int SIGS>
__device__ __forceinline__ double sig_v(int kind, double t) {
    constexpr bool inl = __builtin_popcount(SIGS) <= 2;
    if constexpr (SIGS == S_LIN) return lin_v(t);
    else if constexpr (SIGS == S_SIGMOID) return sigm_v(t);
    else {
        if constexpr ((SIGS & S_LIN) != 0) if (kind == SG_SIGMA_LINEAR) return lin_v(t);
        if constexpr ((SIGS & S_QUAD) != 0) if (kind == SG_SIGMA_QUADRATIC) return quad_v(t);
        if constexpr ((SIGS & S_SIGMOID) != 0) if (kind == SG_SIGMA_SIGMOID) return inl ? sigm_v(t) : sigm_v_call(t);
        if constexpr ((SIGS & S_ERF) != 0) if (kind == SG_SIGMA_ERF) return inl ? erf_v(t) : erf_v_call(t);
        if constexpr ((SIGS & S_SIN) != 0) if (kind == SG_SIGMA_SIN) return inl ? sin_v(t) : sin_v_call(t);
        return 0.0;
    }
}

// sigma(t) and d sigma / d t (derivative of the open piece holding t, 0 outside)
template <int SIGS>
__device__ __forceinline__ void sig_vd(int kind, double t, double& s, double& ds) {
    constexpr bool inl = __builtin_popcount(SIGS) <= 2;
    if constexpr (SIGS == S_LIN) { lin_vd(t, s, ds); return; }
    else if constexpr (SIGS == S_SIGMOID) { sigm_vd(t, s, ds); return; }
    else {
        if constexpr ((SIGS & S_LIN) != 0) if (kind == SG_SIGMA_LINEAR) { lin_vd(t, s, ds); return; }
        if constexpr ((SIGS & S_QUAD) != 0) if (kind == SG_SIGMA_QUADRATIC) { quad_vd(t, s, ds); return; }
        if constexpr ((SIGS & S_SIGMOID) != 0)
            if (kind == SG_SIGMA_SIGMOID) {
                if (inl) { sigm_vd(t, s, ds); } else { const double2 r = sigm_vd_call(t); s = r.x; ds = r.y; }
                return;
            }
        if constexpr ((SIGS & S_ERF) != 0)
            if (kind == SG_SIGMA_ERF) {
                if (inl) { erf_vd(t, s, ds); } else { const double2 r = erf_vd_call(t); s = r.x; ds = r.y; }
                return;
            }
        if constexpr ((SIGS & S_SIN) != 0)
            if (kind == SG_SIGMA_SIN) {
                if (inl) { sin_vd(t, s, ds); } else { const double2 r = sin_vd_call(t); s = r.x; ds = r.y; }
                return;
            }
        s = 0.0;
        ds = 0.0;
    }
}

// d sigma / d t in FP32 (derivative-only uses; the sigma value stays FP64)
__device__ __forceinline__ float sig_d32(int kind, float t) {
    switch (kind) {
        case SG_SIGMA_SIGMOID: {
            if (t <= -(float)kSigmoidCut || t >= (float)kSigmoidCut) return 0.0f;
            const float e = __expf(-fabsf(t));
            const float s = 1.0f / (1.0f + e);
            return s * (1.0f - s);
        }
        case SG_SIGMA_ERF:
            if (t <= -(float)kErfCut || t >= (float)kErfCut) return 0.0f;
            return __expf(-t * t) * (float)kInvSqrtPi;
        case SG_SIGMA_SIN:
            return (t > -(float)kPiHalf && t < (float)kPiHalf) ? 0.5f * __cosf(t) : 0.0f;
        case SG_SIGMA_LINEAR:
            return (t > -0.5f && t < 0.5f) ? 1.0f : 0.0f;
        default:
            if (t > -(float)kInvSqrt2 && t < 0.0f) return 2.0f * ((float)kInvSqrt2 + t);
            if (t >= 0.0f && t < (float)kInvSqrt2) return 2.0f * ((float)kInvSqrt2 - t);
            return 0.0f;
    }
}

// host + device: kind -> bit
__host__ __device__ inline int sigma_bit(int kind) { return 1 << kind; }

__device__ __forceinline__ double kval(int kmode, double k, double width) {
    return kmode == SG_K_LOCAL ? k / width : k;
}

// Rect1D(c; lo, hi) = sigma_k(c - lo) sigma_k(hi - c)
template <int SIGS>
__device__ __forceinline__ double rect_v(int kind, double k, double c, double lo, double hi) {
    return sig_v<SIGS>(kind, k * (c - lo)) * sig_v<SIGS>(kind, k * (hi - c));
}

template <int SIGS>
__device__ __forceinline__ void rect_vd(int kind, double k, double c, double lo, double hi,
                                        double& v, double& dlo, double& dhi) {
    double sa, dsa, sb, dsb;
    sig_vd<SIGS>(kind, k * (c - lo), sa, dsa);
    sig_vd<SIGS>(kind, k * (hi - c), sb, dsb);
    v = sa * sb;
    dlo = -k * dsa * sb;
    dhi = k * sa * dsb;
}

// Largest j in [0, M-2] with xv[j] <= x (or 0), and the position t in [0, 1]
// of x along segment j of a piecewise-linear boundary.
__device__ __forceinline__ void gcart_segment(const double* __restrict__ xv, int M, double x, int& j, double& t) {
    int lo = 0, hi = M - 1;                // invariant: answer in [lo, hi)
    if (x < xv[1]) {
        lo = 0;
    } else if (x >= xv[M - 2]) {
        lo = M - 2;
    } else {
        lo = 1;
        hi = M - 2;                        // xv[lo] <= x < xv[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (xv[mid] <= x) lo = mid; else hi = mid;
        }
    }
    j = lo;
    const double tt = (x - xv[j]) / (xv[j + 1] - xv[j]);
    t = fmin(1.0, fmax(0.0, tt));
}

// Reads through the constant address space: for tables that are constant
// during a kernel and read at a wave-uniform address, the compiler then uses
// scalar loads (through the scalar cache, merged when consecutive).
typedef __attribute__((address_space(4))) const uint32_t* ConstU32;
typedef __attribute__((address_space(4))) const double* ConstF64;
template <class T>
__device__ __forceinline__ T const_space(const void* p) {
    return (T)(uintptr_t)p;
}
// A pointer that is the same in every active lane, moved to scalar registers.
__device__ __forceinline__ const void* uniform_ptr(const void* p) {
    const uint64_t a = (uint64_t)(uintptr_t)p;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)a);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(a >> 32));
    return (const void*)(uintptr_t)(((uint64_t)hi << 32) | lo);
}

// Fourier radius of eq:PSGCboundary at the sample's polar angle about the
// center, R(theta) = R0 - sum_n (c_n cos n theta + s_n sin n theta) (the pi
// shift flips both signs), with cos n theta, sin n theta by repeated rotation
// from cos theta = dx / r, sin theta = dy / r (theta = 0 at the center); and
// the sigma argument k (R - r).  *dR gets d R / d theta when asked for.
__device__ __forceinline__ double polar_arg(const DevPrim& pr, const double* __restrict__ fv, double uc, double vc,
                                            double* r_out = nullptr, double* c1_out = nullptr,
                                            double* s1_out = nullptr, double* dR = nullptr) {
    // called for one primitive at a time by the whole wavefront: its fields
    // sit at a uniform address
    const int N = __builtin_amdgcn_readfirstlane(pr.nvert);
    const ConstF64 f = const_space<ConstF64>(fv + __builtin_amdgcn_readfirstlane(pr.f0));
    const double dx = uc - f[0], dy = vc - f[1];
    const double r2 = dx * dx + dy * dy;
    // one reciprocal square root gives r and the direction cosines (within
    // 2 ulp of sqrt and of the quotients; no FP64 division)
    const double ir = r2 > 0.0 ? rsqrt(r2) : 0.0;
    const double r = r2 * ir;
    const double c1 = r2 > 0.0 ? dx * ir : 1.0, s1 = r2 > 0.0 ? dy * ir : 0.0;
    double R = f[2], d = 0.0, cn = 1.0, sn = 0.0;
    for (int n = 1; n <= N; ++n) {
        const double c = cn * c1 - sn * s1;
        sn = sn * c1 + cn * s1;
        cn = c;
        const double a = f[2 + n], b = f[2 + N + n];
        R -= a * cn + b * sn;
        d += (double)n * (a * sn - b * cn);
    }
    if (r_out) *r_out = r;
    if (c1_out) *c1_out = c1;
    if (s1_out) *s1_out = s1;
    if (dR) *dR = d;
    return pr.k0 * (R - r);
}

// Polar2D (Tab. autodiffgeo): the radius R (1 + delta cos(alpha theta)) about
// (x0, y0), cos(alpha theta) by alpha rotations from (dx, dy) / r (theta = 0 at
// the center); the sigma argument k (R(theta) - r).
__device__ __forceinline__ double polar2d_arg(const DevPrim& pr, const double* __restrict__ fv, double uc,
                                              double vc) {
    // called for one primitive at a time by the whole wavefront: its fields
    // sit at a uniform address
    const int A = __builtin_amdgcn_readfirstlane(pr.nvert);
    const ConstF64 f = const_space<ConstF64>(fv + __builtin_amdgcn_readfirstlane(pr.f0));
    const double dx = uc - f[0], dy = vc - f[1];
    const double r2 = dx * dx + dy * dy;
    const double ir = r2 > 0.0 ? rsqrt(r2) : 0.0;
    const double r = r2 * ir;
    const double c1 = r2 > 0.0 ? dx * ir : 1.0, s1 = r2 > 0.0 ? dy * ir : 0.0;
    double cn = 1.0, sn = 0.0;
    for (int n = 0; n < A; ++n) {
        const double c = cn * c1 - sn * s1;
        sn = sn * c1 + cn * s1;
        cn = c;
    }
    return pr.k0 * (f[2] * (1.0 + f[3] * cn) - r);
}

// Half-width f(x) of the taper's sine-series boundary (eq:taper_boundary):
// phi = pi (x - x0) / L, sin i phi by repeated rotation from (cos phi, sin phi),
// envelope 0.1 + 0.45 (1 - cos 2 phi) = 0.1 + 0.9 sin^2 phi.  cst: x0 L w_in w_out yc.
__device__ __forceinline__ double series_f(const DevPrim& pr, const double* __restrict__ fv,
                                           const double* __restrict__ cst, double uc, double* env_out = nullptr,
                                           double* s1_out = nullptr, double* c1_out = nullptr) {
    // called for one primitive at a time by the whole wavefront: its fields
    // and constants sit at uniform addresses
    const ConstF64 cc = const_space<ConstF64>(uniform_ptr(cst));
    const double x0 = cc[0], L = cc[1], w_in = cc[2], w_out = cc[3];
    const double u = (uc - x0) / L;
    double s1, c1;
    sincospi(u, &s1, &c1);
    const double env = 0.1 + 0.9 * s1 * s1;
    const ConstF64 v = const_space<ConstF64>(fv + __builtin_amdgcn_readfirstlane(pr.f0) + 2);
    const int K = __builtin_amdgcn_readfirstlane(pr.nvert);
    double sum = 0.0, si = s1, ci = c1;
#pragma unroll 8
    for (int i = 0; i < K; ++i) {
        sum += v[i] * si;
        const double sn = si * c1 + ci * s1;
        ci = ci * c1 - si * s1;
        si = sn;
    }
    if (env_out) *env_out = env;
    if (s1_out) *s1_out = s1;
    if (c1_out) *c1_out = c1;
    return 0.5 * w_in + 0.5 * (w_out - w_in) * u + env * sum;
}

// In-plane factor F(u, v) of a primitive (value only).  gs: the sample's entry
// of the primitive's segment table (piecewise-linear boundaries only).
template <int TYPES, int SIGS>
__device__ __forceinline__ double prim_value(const DevPrim& pr, const double* __restrict__ fv,
                                             const double* __restrict__ cst,
                                             double uc, double uw, double vc, double vw, const GSeg* gs) {
    if constexpr ((TYPES & T_BOX) != 0) {
        if (TYPES == T_BOX || pr.type == SG_PRIM_BOX) {
            double f = 1.0;
            if (pr.ubnd) f = rect_v<SIGS>(pr.sk0, kval(pr.sm0, pr.k0, uw), uc, fv[pr.fu0], fv[pr.fu1]);
            if (pr.vbnd) f *= rect_v<SIGS>(pr.sk1, kval(pr.sm1, pr.k1, vw), vc, fv[pr.fv0], fv[pr.fv1]);
            return f;
        }
    }
    if constexpr ((TYPES & T_ELL) != 0) {
        if (pr.type == SG_PRIM_ELLIPSE) {
            const double dx = (uc - fv[pr.f0]) * pr.iax, dy = (vc - fv[pr.f0 + 1]) * pr.iay;
            const double rho2 = dx * dx + dy * dy;
            const double r = fv[pr.f0 + 2];
            const double rhi = r + pr.reach0, rlo = r - pr.reach0;
            if (rhi <= 0.0 || rho2 >= rhi * rhi) return 0.0;      // beyond the sigma support
            if (rlo > 0.0 && rho2 <= rlo * rlo) return 1.0;
            return sig_v<SIGS>(pr.sk0, pr.k0 * (r - sqrt(rho2)));
        }
    }
    if constexpr ((TYPES & T_POLY) != 0) {
        if (pr.type == SG_PRIM_POLY) {
            // one primitive at a time for the whole wavefront: scalar loads
            const int N = __builtin_amdgcn_readfirstlane(pr.nvert);
            const ConstF64 xs = const_space<ConstF64>(fv + __builtin_amdgcn_readfirstlane(pr.f0));
            const ConstF64 ys = xs + N;
            double f = 1.0;
            for (int i = 0; i < N && f > 0.0; ++i) {
                const int j = (i + 1 == N) ? 0 : i + 1;
                const double ex = xs[j] - xs[i], ey = ys[j] - ys[i];
                const double L = sqrt(ex * ex + ey * ey);
                const double d = (ex * (vc - ys[i]) - ey * (uc - xs[i])) / L;
                f *= sig_v<SIGS>(pr.sk0, pr.k0 * d);
            }
            return f;
        }
    }
    if constexpr ((TYPES & T_GCART) != 0) {
        if (pr.type == SG_PRIM_GCART) {
            const int M = pr.nvert;
            const double rx = rect_v<SIGS>(pr.sk0, kval(pr.sm0, pr.k0, uw), uc, fv[pr.f0], fv[pr.f0 + 1]);
            if (rx == 0.0) return 0.0;
            const GSeg sgm = *gs;
            const int j = sgm.j;
            const double t = sgm.t;
            const double* yp = fv + pr.f0 + 2;
            const double* ym = yp + M;
            const double fp = (1.0 - t) * yp[j] + t * yp[j + 1];
            const double fm = (1.0 - t) * ym[j] + t * ym[j + 1];
            const double ky = kval(pr.sm1, pr.k1, vw);
            return rx * sig_v<SIGS>(pr.sk1, ky * (fp - vc)) * sig_v<SIGS>(pr.sk1, ky * (vc - fm));
        }
    }
    if constexpr ((TYPES & T_POLAR) != 0) {
        if (pr.type == SG_PRIM_POLAR) return sig_v<SIGS>(pr.sk0, polar_arg(pr, fv, uc, vc));
        if (pr.type == SG_PRIM_POLAR2D) return sig_v<SIGS>(pr.sk0, polar2d_arg(pr, fv, uc, vc));
    }
    if constexpr ((TYPES & T_SERIES) != 0) {
        if (pr.type == SG_PRIM_SERIES) {
            const double rx = rect_v<SIGS>(pr.sk0, kval(pr.sm0, pr.k0, uw), uc, fv[pr.f0], fv[pr.f0 + 1]);
            if (rx == 0.0) return 0.0;
            const double* c = cst + pr.c0;
            const double f = series_f(pr, fv, c, uc);
            const double ky = kval(pr.sm1, pr.k1, vw), yr = vc - c[4];
            return rx * sig_v<SIGS>(pr.sk1, ky * (f - yr)) * sig_v<SIGS>(pr.sk1, ky * (f + yr));
        }
    }
    return 0.0;
}

// ---- where the in-plane derivatives can be nonzero (sparse reverse mode)
// d sigma / d t vanishes outside |t| < sigma_cut(kind) for every kind; the
// slack covers evaluation-order differences between the value code here and
// the partials code, so a sample is never taken as dead where a partial is
// nonzero.
constexpr double kSupportSlack = 1e-9;
template <int SIGS>
__device__ __forceinline__ bool sig_live(int kind, double t, double slack = kSupportSlack) {
    if constexpr (SIGS == S_LIN) return fabs(t) < 0.5 + slack;
    else return fabs(t) < sigma_cut(kind) + slack;
}
// The Fourier-radius partials evaluate their argument in FP32 (error up to
// ~1e-5 in t for order-6 radii): their probe takes a wider slack.
constexpr double kSupportSlack32 = 1e-3;

// prim_value of a polygon or a piecewise-linear boundary, and in *live
// whether some in-plane partial of the primitive can be nonzero at the sample:
// a partial with respect to one sigma argument is that argument's sigma'
// times the product of the other factors, so it needs the argument inside
// its support and every other factor nonzero.  The value is the one
// prim_value returns (same operations, no early exits).
template <int TYPES, int SIGS>
__device__ __forceinline__ double prim_value_live(const DevPrim& pr, const double* __restrict__ fv,
                                                  const double* __restrict__ cst,
                                                  double uc, double uw, double vc, double vw, const GSeg* gs,
                                                  bool& live) {
    if constexpr ((TYPES & T_POLY) != 0) {
        if (pr.type == SG_PRIM_POLY) {
            // one primitive at a time for the whole wavefront: scalar loads
            const int N = __builtin_amdgcn_readfirstlane(pr.nvert);
            const ConstF64 xs = const_space<ConstF64>(fv + __builtin_amdgcn_readfirstlane(pr.f0));
            const ConstF64 ys = xs + N;
            double f = 1.0;
            int nzero = 0;
            bool any = false, zlive = false;
            for (int i = 0; i < N; ++i) {
                const int j = (i + 1 == N) ? 0 : i + 1;
                const double ex = xs[j] - xs[i], ey = ys[j] - ys[i];
                const double L = sqrt(ex * ex + ey * ey);
                const double t = pr.k0 * ((ex * (vc - ys[i]) - ey * (uc - xs[i])) / L);
                const double sv = sig_v<SIGS>(pr.sk0, t);
                const bool l = sig_live<SIGS>(pr.sk0, t);
                if (sv == 0.0) {
                    ++nzero;
                    zlive = l;
                }
                any = any || l;
                f *= sv;
            }
            live = (nzero == 0) ? any : (nzero == 1 && zlive);
            return f;
        }
    }
    if constexpr ((TYPES & T_GCART) != 0) {
        if (pr.type == SG_PRIM_GCART) {
            const int M = pr.nvert;
            const double kx = kval(pr.sm0, pr.k0, uw);
            const double ta = kx * (uc - fv[pr.f0]), tb = kx * (fv[pr.f0 + 1] - uc);
            const double rx = sig_v<SIGS>(pr.sk0, ta) * sig_v<SIGS>(pr.sk0, tb);
            const GSeg sgm = *gs;
            const int j = sgm.j;
            const double t = sgm.t;
            const double* yp = fv + pr.f0 + 2;
            const double* ym = yp + M;
            const double fp = (1.0 - t) * yp[j] + t * yp[j + 1];
            const double fm = (1.0 - t) * ym[j] + t * ym[j + 1];
            const double ky = kval(pr.sm1, pr.k1, vw);
            const double tp = ky * (fp - vc), tm = ky * (vc - fm);
            const double sp = sig_v<SIGS>(pr.sk1, tp), sm = sig_v<SIGS>(pr.sk1, tm);
            const bool lx = sig_live<SIGS>(pr.sk0, ta) || sig_live<SIGS>(pr.sk0, tb);
            live = (lx && sp * sm != 0.0) ||
                   (rx != 0.0 && ((sig_live<SIGS>(pr.sk1, tp) && sm != 0.0) || (sig_live<SIGS>(pr.sk1, tm) && sp != 0.0)));
            return rx * sp * sm;
        }
    }
    if constexpr ((TYPES & T_POLAR) != 0) {
        if (pr.type == SG_PRIM_POLAR || pr.type == SG_PRIM_POLAR2D) {
            const double t = pr.type == SG_PRIM_POLAR ? polar_arg(pr, fv, uc, vc) : polar2d_arg(pr, fv, uc, vc);
            live = sig_live<SIGS>(pr.sk0, t, kSupportSlack32);
            return sig_v<SIGS>(pr.sk0, t);
        }
    }
    if constexpr ((TYPES & T_SERIES) != 0) {
        if (pr.type == SG_PRIM_SERIES) {
            // same factors and operations as prim_value; the partials follow the GCART pattern
            const double kx = kval(pr.sm0, pr.k0, uw);
            const double ta = kx * (uc - fv[pr.f0]), tb = kx * (fv[pr.f0 + 1] - uc);
            const double rx = sig_v<SIGS>(pr.sk0, ta) * sig_v<SIGS>(pr.sk0, tb);
            const double* c = cst + pr.c0;
            const double f = series_f(pr, fv, c, uc);
            const double ky = kval(pr.sm1, pr.k1, vw), yr = vc - c[4];
            const double tp = ky * (f - yr), tm = ky * (f + yr);
            const double sp = sig_v<SIGS>(pr.sk1, tp), sm = sig_v<SIGS>(pr.sk1, tm);
            const bool lx = sig_live<SIGS>(pr.sk0, ta) || sig_live<SIGS>(pr.sk0, tb);
            live = (lx && sp * sm != 0.0) ||
                   (rx != 0.0 && ((sig_live<SIGS>(pr.sk1, tp) && sm != 0.0) || (sig_live<SIGS>(pr.sk1, tm) && sp != 0.0)));
            return rx == 0.0 ? 0.0 : rx * sp * sm;
        }
    }
    live = false;
    return 0.0;
}

}  // namespace sg

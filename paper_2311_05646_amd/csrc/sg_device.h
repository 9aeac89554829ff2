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

// sigma(t)
__device__ __forceinline__ double sig_v(int kind, double t) {
    switch (kind) {
        case SG_SIGMA_SIGMOID:
            if (t <= -kSigmoidCut) return 0.0;
            if (t >= kSigmoidCut) return 1.0;
            return 1.0 / (1.0 + exp(-t));
        case SG_SIGMA_ERF:
            if (t <= -kErfCut) return 0.0;
            if (t >= kErfCut) return 1.0;
            return 0.5 * (1.0 + erf(t));
        case SG_SIGMA_SIN:
            if (t < -kPiHalf) return 0.0;
            if (t > kPiHalf) return 1.0;
            return 0.5 * (1.0 + sin(t));
        case SG_SIGMA_LINEAR:
            return fmax(0.0, fmin(1.0, t + 0.5));
        default: {  // quadratic
            if (t < -kInvSqrt2) return 0.0;
            if (t < 0.0) { const double a = kInvSqrt2 + t; return a * a; }
            if (t <= kInvSqrt2) { const double a = kInvSqrt2 - t; return 1.0 - a * a; }
            return 1.0;
        }
    }
}

// sigma(t) and d sigma / d t (derivative of the open piece holding t, 0 outside)
__device__ __forceinline__ void sig_vd(int kind, double t, double& s, double& ds) {
    switch (kind) {
        case SG_SIGMA_SIGMOID:
            if (t <= -kSigmoidCut) { s = 0.0; ds = 0.0; return; }
            if (t >= kSigmoidCut) { s = 1.0; ds = 0.0; return; }
            s = 1.0 / (1.0 + exp(-t));
            ds = s * (1.0 - s);
            return;
        case SG_SIGMA_ERF:
            if (t <= -kErfCut) { s = 0.0; ds = 0.0; return; }
            if (t >= kErfCut) { s = 1.0; ds = 0.0; return; }
            s = 0.5 * (1.0 + erf(t));
            ds = exp(-t * t) * kInvSqrtPi;
            return;
        case SG_SIGMA_SIN:
            if (t < -kPiHalf) { s = 0.0; ds = 0.0; return; }
            if (t > kPiHalf) { s = 1.0; ds = 0.0; return; }
            {
                double sn, cs;
                sincos(t, &sn, &cs);
                s = 0.5 * (1.0 + sn);
                ds = (t > -kPiHalf && t < kPiHalf) ? 0.5 * cs : 0.0;
            }
            return;
        case SG_SIGMA_LINEAR:
            s = fmax(0.0, fmin(1.0, t + 0.5));
            ds = (t > -0.5 && t < 0.5) ? 1.0 : 0.0;
            return;
        default:
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
            return;
    }
}

__device__ __forceinline__ double kval(int kmode, double k, double width) {
    return kmode == SG_K_LOCAL ? k / width : k;
}

// Rect1D(c; lo, hi) = sigma_k(c - lo) sigma_k(hi - c)
__device__ __forceinline__ double rect_v(int kind, double k, double c, double lo, double hi) {
    return sig_v(kind, k * (c - lo)) * sig_v(kind, k * (hi - c));
}

__device__ __forceinline__ void rect_vd(int kind, double k, double c, double lo, double hi,
                                        double& v, double& dlo, double& dhi) {
    double sa, dsa, sb, dsb;
    sig_vd(kind, k * (c - lo), sa, dsa);
    sig_vd(kind, k * (hi - c), sb, dsb);
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

// In-plane factor F(u, v) of a primitive (value only).
__device__ __forceinline__ double prim_value(const DevPrim& pr, const double* __restrict__ fv,
                                             const double* __restrict__ cst,
                                             double uc, double uw, double vc, double vw) {
    switch (pr.type) {
        case SG_PRIM_BOX: {
            double f = 1.0;
            if (pr.ubnd) f = rect_v(pr.sk0, kval(pr.sm0, pr.k0, uw), uc, fv[pr.fu0], fv[pr.fu1]);
            if (pr.vbnd) f *= rect_v(pr.sk1, kval(pr.sm1, pr.k1, vw), vc, fv[pr.fv0], fv[pr.fv1]);
            return f;
        }
        case SG_PRIM_ELLIPSE: {
            const double dx = (uc - fv[pr.f0]) / pr.ax, dy = (vc - fv[pr.f0 + 1]) / pr.ay;
            const double rho = sqrt(dx * dx + dy * dy);
            return sig_v(pr.sk0, pr.k0 * (fv[pr.f0 + 2] - rho));
        }
        case SG_PRIM_POLY: {
            const int N = pr.nvert;
            const double* xs = fv + pr.f0;
            const double* ys = xs + N;
            double f = 1.0;
            for (int i = 0; i < N && f > 0.0; ++i) {
                const int j = (i + 1 == N) ? 0 : i + 1;
                const double ex = xs[j] - xs[i], ey = ys[j] - ys[i];
                const double L = sqrt(ex * ex + ey * ey);
                const double d = (ex * (vc - ys[i]) - ey * (uc - xs[i])) / L;
                f *= sig_v(pr.sk0, pr.k0 * d);
            }
            return f;
        }
        default: {  // GCART
            const int M = pr.nvert;
            const double rx = rect_v(pr.sk0, kval(pr.sm0, pr.k0, uw), uc, fv[pr.f0], fv[pr.f0 + 1]);
            if (rx == 0.0) return 0.0;
            int j;
            double t;
            gcart_segment(cst + pr.c0, M, uc, j, t);
            const double* yp = fv + pr.f0 + 2;
            const double* ym = yp + M;
            const double fp = (1.0 - t) * yp[j] + t * yp[j + 1];
            const double fm = (1.0 - t) * ym[j] + t * ym[j + 1];
            const double ky = kval(pr.sm1, pr.k1, vw);
            return rx * sig_v(pr.sk1, ky * (fp - vc)) * sig_v(pr.sk1, ky * (vc - fm));
        }
    }
}

}  // namespace sg

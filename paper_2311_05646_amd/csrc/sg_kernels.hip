// gfx950 kernels of the shape-gradient path.
//
//  k_stage   p -> resolved primitive fields (a + b p[idx]), support boxes and
//            the per-class extrusion tables Z(w), dZ/dlo, dZ/dhi; zeroes the
//            gradient accumulator.
//  k_column  one thread per in-plane sample (u, v) of one component, walking
//            a segment of its column (w).  In-plane factors F_h of the
//            candidate primitives are computed once per column in FP64; each
//            column step composes the classes (eq:union, eq:intersection,
//            difference) and either stores eps (MODE_EPS), stores the FD
//            difference plane (MODE_FD), or accumulates the reverse-mode
//            column sums A_c = sum_w g * d eps / d s_c * Z_c(w) (MODE_VJP_*),
//            with g = 2 omega Im(E Eadj) (eq:1) or an upstream dF/deps.  After
//            the column the in-plane partials are multiplied by A_c and
//            reduced across the wavefront; lane 0 adds one FP64 atomic per
//            parameter field touched by the wavefront.
//  k_gplane  g = 2 omega Im(E Eadj) plane (finite-difference baseline)
//  k_dot     sum a * b (finite-difference baseline reduction)
#include "sg_device.h"

namespace sg {

// ------------------------------------------------------------------ stage
__global__ __launch_bounds__(256) void k_stage(const StageParams sp) {
    const int var = blockIdx.y;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const double delta = sp.delta[var];
    auto resolve = [&](int f) -> double {
        const sg_field r = sp.fref[f];
        if (r.idx < 0) return r.a;
        double pv = sp.p[r.idx];
        if (r.idx == sp.pert_idx) pv += delta;
        return r.a + r.b * pv;
    };
    if (var == 0 && sp.zero_ptr != nullptr && t < sp.zero_n) sp.zero_ptr[t] = 0.0;
    if (t < sp.nprim) {
        const DevPrim pr = sp.prims[t];
        double* fv = sp.fval[var];
        int nf;
        switch (pr.type) {
            case SG_PRIM_BOX: nf = 6; break;
            case SG_PRIM_ELLIPSE: nf = 5; break;
            case SG_PRIM_POLY: nf = 2 * pr.nvert + 2; break;
            default: nf = 2 * pr.nvert + 4; break;
        }
        for (int i = 0; i < nf; ++i) fv[pr.f0 + i] = resolve(pr.f0 + i);
        const double inf = __builtin_huge_val();
        double4 b = make_double4(-inf, inf, -inf, inf);
        if (pr.type == SG_PRIM_BOX) {
            if (pr.ubnd) { b.x = resolve(pr.fu0) - pr.reach0; b.y = resolve(pr.fu1) + pr.reach0; }
            if (pr.vbnd) { b.z = resolve(pr.fv0) - pr.reach1; b.w = resolve(pr.fv1) + pr.reach1; }
        } else if (pr.type == SG_PRIM_ELLIPSE) {
            const double R = resolve(pr.f0 + 2) + pr.reach0;
            const double x0 = resolve(pr.f0), y0 = resolve(pr.f0 + 1);
            if (R < 0.0) {
                b = make_double4(inf, -inf, inf, -inf);
            } else {
                b = make_double4(x0 - R * pr.ax, x0 + R * pr.ax, y0 - R * pr.ay, y0 + R * pr.ay);
            }
        } else if (pr.type == SG_PRIM_POLY) {
            // the support is the polygon offset outward by reach0: its vertices
            // are v_i - d (n_{i-1} + n_i) / (1 + n_{i-1} . n_i), n inward normals
            const int N = pr.nvert;
            b = make_double4(inf, -inf, inf, -inf);
            for (int i = 0; i < N; ++i) {
                const int ip = (i == 0) ? N - 1 : i - 1, in = (i + 1 == N) ? 0 : i + 1;
                const double xi = resolve(pr.f0 + i), yi = resolve(pr.f0 + N + i);
                const double xp = resolve(pr.f0 + ip), yp = resolve(pr.f0 + N + ip);
                const double xn = resolve(pr.f0 + in), yn = resolve(pr.f0 + N + in);
                double ax = xi - xp, ay = yi - yp, bx = xn - xi, by = yn - yi;
                const double la = sqrt(ax * ax + ay * ay), lb = sqrt(bx * bx + by * by);
                const double nax = -ay / la, nay = ax / la, nbx = -by / lb, nby = bx / lb;
                const double den = 1.0 + nax * nbx + nay * nby;
                double ox, oy;
                if (den > 1e-12) {
                    ox = xi - pr.reach0 * (nax + nbx) / den;
                    oy = yi - pr.reach0 * (nay + nby) / den;
                    b.x = fmin(b.x, ox); b.y = fmax(b.y, ox);
                    b.z = fmin(b.z, oy); b.w = fmax(b.w, oy);
                } else {
                    b = make_double4(-inf, inf, -inf, inf);
                    break;
                }
            }
        } else {  // GCART
            const int M = pr.nvert;
            b.x = resolve(pr.f0) - pr.reach0;
            b.y = resolve(pr.f0 + 1) + pr.reach0;
            double ymax = -inf, ymin = inf;
            for (int j = 0; j < M; ++j) {
                ymax = fmax(ymax, resolve(pr.f0 + 2 + j));
                ymin = fmin(ymin, resolve(pr.f0 + 2 + M + j));
            }
            b.z = ymin - pr.reach1;
            b.w = ymax + pr.reach1;
        }
        sp.bbox[var][t] = b;
    }
    const int64_t nz = (int64_t)sp.ncomp * sp.nclass * sp.nw;
    if (t < nz) {
        const int w = (int)(t % sp.nw);
        const int c = (int)((t / sp.nw) % sp.nclass);
        const int comp = (int)(t / ((int64_t)sp.nw * sp.nclass));
        const DevClass cl = sp.cls[c];
        double z = 1.0, dlo = 0.0, dhi = 0.0;
        if (cl.bounded) {
            const double wc = sp.wc[comp][w], wwid = sp.ww[comp][w];
            const double k = kval(cl.smode, cl.k, wwid);
            rect_vd<S_ALL>(cl.skind, k, wc, resolve(cl.flo), resolve(cl.fhi), z, dlo, dhi);
        }
        double* zt = sp.ztab[var] + 3 * t;
        zt[0] = z;
        zt[1] = dlo;
        zt[2] = dhi;
    }
}

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Adds the wavefront sum of v (one value per lane) times the field's scale to
// grad[field's parameter].  Called with wave-uniform control flow.
__device__ __forceinline__ void emit(const KParams& P, int field, float v) {
    const sg_field r = P.fref[field];
    if (r.idx < 0) return;
    if (__ballot(v != 0.0f) == 0) return;
    const float s = wave_sum(v);
    if ((threadIdx.x & 63) == 0) atomicAdd(P.grad + r.idx, r.b * (double)s);
}

__device__ __forceinline__ void add_field(const KParams& P, int field, float v) {
    const sg_field r = P.fref[field];
    if (r.idx >= 0 && v != 0.0f) atomicAdd(P.grad + r.idx, r.b * (double)v);
}

// Appends (in primitive order) every primitive whose support box meets the
// tile [ulo, uhi] x [vlo, vhi] to s_cand, scanning from `start` until the list
// could overflow.  Returns the count; *next = first primitive not scanned.
__device__ int build_list(const double4* __restrict__ bb, int nprim, int start, double ulo, double uhi,
                          double vlo, double vhi, int* s_cand, int* s_cnt, int* next) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int n = 0;
    int base = start;
    for (; base < nprim && n + kBlock <= kCandCap; base += kBlock) {
        const int i = base + tid;
        bool hit = false;
        if (i < nprim) {
            const double4 b = bb[i];
            hit = (b.x <= uhi) && (b.y >= ulo) && (b.z <= vhi) && (b.w >= vlo);
        }
        const uint64_t m = __ballot(hit);
        if (lane == 0) s_cnt[wave] = __popcll(m);
        __syncthreads();
        int off = n, tot = 0;
#pragma unroll
        for (int q = 0; q < kBlock / 64; ++q) {
            const int cq = s_cnt[q];
            if (q < wave) off += cq;
            tot += cq;
        }
        if (hit) s_cand[off + __popcll(m & ((1ull << lane) - 1ull))] = i;
        n += tot;
        __syncthreads();
    }
    *next = base;
    return n;
}

struct Tile {
    double ulo, uhi, vlo, vhi;      // block: centers of the first / last sample
    double wulo, wuhi, wvlo, wvhi;  // this wavefront
    bool wave_live;
};

__device__ __forceinline__ bool wave_meets(const Tile& T, const double4 b) {
    return (b.x <= T.wuhi) && (b.y >= T.wulo) && (b.z <= T.wvhi) && (b.w >= T.wvlo);
}

template <int NC>
__device__ __forceinline__ void add_to_class(double (&F)[NC], int cls, double v) {
#pragma unroll
    for (int c = 0; c < NC; ++c)
        if (c == cls) F[c] += v;
}

// Sum of F_h over the candidates, per class, at (uc, vc).
template <int NC, int TYPES, int SIGS>
__device__ void inplane_sums(const KParams& P, const double4* __restrict__ bbox, const double* __restrict__ fval,
                             const Tile& T, double uc, double uw, double vc, double vw, int* s_cand, int* s_cnt,
                             double (&F)[NC], int& nlist, bool& complete) {
#pragma unroll
    for (int c = 0; c < NC; ++c) F[c] = 0.0;
    int next = 0;
    bool first = true;
    while (first || next < P.nprim) {
        if (!first) __syncthreads();
        const int n = build_list(bbox, P.nprim, next, T.ulo, T.uhi, T.vlo, T.vhi, s_cand, s_cnt, &next);
        if (first) { complete = next >= P.nprim; nlist = n; }
        first = false;
        if (!T.wave_live) continue;
        for (int j = 0; j < n; ++j) {
            const int pi = uniform_int(s_cand[j]);
            if (!wave_meets(T, bbox[pi])) continue;
            const DevPrim pr = P.prims[pi];
            const double f = prim_value<TYPES, SIGS>(pr, fval, P.consts, uc, uw, vc, vw);
            add_to_class(F, pr.cls, f);
        }
    }
}

// Composition at one column step: root value s and, per group g, the
// derivative r_g = d s / d (group sum g) in {0, +1, -1}.
struct Comp {
    double s;
    double r0, r1, r2, r3;
};

__device__ __forceinline__ void group_op(const KParams& P, int g, double S, double& val, double& msk) {
    if (P.group_op[g] == SG_OP_INTERSECTION) {
        const double nm1 = P.group_nm1[g];
        val = fmax(nm1, S) - nm1;
        msk = (S > nm1) ? 1.0 : 0.0;
    } else {
        val = fmin(1.0, S);
        msk = (S < 1.0) ? 1.0 : 0.0;
    }
}

template <int NC>
__device__ __forceinline__ Comp compose(const KParams& P, const double (&F)[NC], const double* __restrict__ zt,
                                        double (&Z)[NC]) {
    double S0 = 0.0, S1 = 0.0, S2 = 0.0, S3 = 0.0;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        if (c < P.nclass) {
            Z[c] = zt[3 * c * P.nw];
            const double t = F[c] * Z[c];
            const int g = P.cls_group[c];
            if (g == 0) S0 += t;
            else if (g == 1) S1 += t;
            else if (g == 2) S2 += t;
            else S3 += t;
        } else {
            Z[c] = 0.0;
        }
    }
    double v0, v1 = 0.0, v2 = 0.0, v3 = 0.0, m0, m1 = 0.0, m2 = 0.0, m3 = 0.0;
    group_op(P, 0, S0, v0, m0);
    if (P.ngroup > 1) group_op(P, 1, S1, v1, m1);
    if (P.ngroup > 2) group_op(P, 2, S2, v2, m2);
    if (P.ngroup > 3) group_op(P, 3, S3, v3, m3);
    Comp o;
    if (P.root_op == ROOT_NONE) {
        o.s = v0;
        o.r0 = m0;
        o.r1 = o.r2 = o.r3 = 0.0;
    } else if (P.root_op == SG_OP_DIFFERENCE) {
        const double d = v0 - v1;
        o.s = fmax(0.0, d);
        const double m = d > 0.0 ? 1.0 : 0.0;
        o.r0 = m * m0;
        o.r1 = -m * m1;
        o.r2 = o.r3 = 0.0;
    } else {
        const double tot = v0 + v1 + v2 + v3;
        double m;
        if (P.root_op == SG_OP_UNION) {
            o.s = fmin(1.0, tot);
            m = tot < 1.0 ? 1.0 : 0.0;
        } else {
            o.s = fmax(P.root_nm1, tot) - P.root_nm1;
            m = tot > P.root_nm1 ? 1.0 : 0.0;
        }
        o.r0 = m * m0;
        o.r1 = m * m1;
        o.r2 = m * m2;
        o.r3 = m * m3;
    }
    return o;
}

template <int NC>
__device__ __forceinline__ float class_pick(const float (&A)[NC], int cls) {
    float a = 0.0f;
#pragma unroll
    for (int c = 0; c < NC; ++c)
        if (c == cls) a = A[c];
    return a;
}

// In-plane partials of one primitive times its class column sum a, reduced
// over the wavefront and added to the gradient.
template <int TYPES, int SIGS>
__device__ void emit_partials(const KParams& P, const DevPrim& pr, int pi, float a, double uc, double uw,
                              double vc, double vw) {
    const double* fv = P.fval;
    const double ad = (double)a;
    const int type = (TYPES == T_BOX) ? SG_PRIM_BOX : pr.type;
    switch (type) {
        case SG_PRIM_BOX: {
            if constexpr ((TYPES & T_BOX) == 0) break;
            double ru = 1.0, du0 = 0.0, du1 = 0.0, rv = 1.0, dv0 = 0.0, dv1 = 0.0;
            if (pr.ubnd) rect_vd<SIGS>(pr.sk0, kval(pr.sm0, pr.k0, uw), uc, fv[pr.fu0], fv[pr.fu1], ru, du0, du1);
            if (pr.vbnd) rect_vd<SIGS>(pr.sk1, kval(pr.sm1, pr.k1, vw), vc, fv[pr.fv0], fv[pr.fv1], rv, dv0, dv1);
            if (pr.ubnd) {
                emit(P, pr.fu0, (float)(ad * du0 * rv));
                emit(P, pr.fu1, (float)(ad * du1 * rv));
            }
            if (pr.vbnd) {
                emit(P, pr.fv0, (float)(ad * ru * dv0));
                emit(P, pr.fv1, (float)(ad * ru * dv1));
            }
            break;
        }
        case SG_PRIM_ELLIPSE: {
            if constexpr ((TYPES & T_ELL) == 0) break;
            const double dx = uc - fv[pr.f0], dy = vc - fv[pr.f0 + 1];
            const double qx = dx / pr.ax, qy = dy / pr.ay;
            const double rho = sqrt(qx * qx + qy * qy);
            double s, ds;
            sig_vd<SIGS>(pr.sk0, pr.k0 * (fv[pr.f0 + 2] - rho), s, ds);
            const double g = ad * pr.k0 * ds;  // a * dF / d(r - rho)
            const double inv = rho > 0.0 ? 1.0 / rho : 0.0;
            emit(P, pr.f0, (float)(g * qx * inv / pr.ax));       // -drho/dx0 = dx / (ax^2 rho)
            emit(P, pr.f0 + 1, (float)(g * qy * inv / pr.ay));
            emit(P, pr.f0 + 2, (float)g);
            break;
        }
        case SG_PRIM_POLY: {
            if constexpr ((TYPES & T_POLY) == 0) break;
            const int N = pr.nvert;
            const double* xs = fv + pr.f0;
            const double* ys = xs + N;
            double pnz = 1.0;
            int nzero = 0, zidx = -1;
            for (int i = 0; i < N; ++i) {
                const int j = (i + 1 == N) ? 0 : i + 1;
                const double ex = xs[j] - xs[i], ey = ys[j] - ys[i];
                const double L = sqrt(ex * ex + ey * ey);
                const double sv = sig_v<SIGS>(pr.sk0, pr.k0 * (ex * (vc - ys[i]) - ey * (uc - xs[i])) / L);
                if (sv == 0.0) { ++nzero; zidx = i; } else { pnz *= sv; }
            }
            for (int i = 0; i < N; ++i) {
                const int j = (i + 1 == N) ? 0 : i + 1;
                const double ex = xs[j] - xs[i], ey = ys[j] - ys[i];
                const double L = sqrt(ex * ex + ey * ey);
                const double wx = uc - xs[i], wy = vc - ys[i];
                const double d = (ex * wy - ey * wx) / L;
                double s, ds;
                sig_vd<SIGS>(pr.sk0, pr.k0 * d, s, ds);
                double other;
                if (nzero == 0) other = pnz / s;
                else if (nzero == 1 && zidx == i) other = pnz;
                else other = 0.0;
                const double g = ad * pr.k0 * ds * other;   // a * dF / d d_i
                const double iL = 1.0 / L, dL2 = d * iL * iL;
                emit(P, pr.f0 + i, (float)(g * ((ey - wy) * iL + dL2 * ex)));
                emit(P, pr.f0 + N + i, (float)(g * ((wx - ex) * iL + dL2 * ey)));
                emit(P, pr.f0 + j, (float)(g * (wy * iL - dL2 * ex)));
                emit(P, pr.f0 + N + j, (float)(g * (-wx * iL - dL2 * ey)));
            }
            break;
        }
        default: {  // GCART
            if constexpr ((TYPES & T_GCART) == 0) break;
            const int M = pr.nvert;
            double rx, drx0, drx1;
            rect_vd<SIGS>(pr.sk0, kval(pr.sm0, pr.k0, uw), uc, fv[pr.f0], fv[pr.f0 + 1], rx, drx0, drx1);
            int j;
            double t;
            gcart_segment(P.consts + pr.c0, M, uc, j, t);
            const double* yp = fv + pr.f0 + 2;
            const double* ym = yp + M;
            const double fp = (1.0 - t) * yp[j] + t * yp[j + 1];
            const double fm = (1.0 - t) * ym[j] + t * ym[j + 1];
            const double ky = kval(pr.sm1, pr.k1, vw);
            double sp, dsp, sm, dsm;
            sig_vd<SIGS>(pr.sk1, ky * (fp - vc), sp, dsp);
            sig_vd<SIGS>(pr.sk1, ky * (vc - fm), sm, dsm);
            const double fy = sp * sm;
            emit(P, pr.f0, (float)(ad * drx0 * fy));
            emit(P, pr.f0 + 1, (float)(ad * drx1 * fy));
            const double gp = ad * rx * ky * dsp * sm;    // a * dF / d f+
            const double gm = -ad * rx * sp * ky * dsm;   // a * dF / d f-
            float c0 = (float)(gp * (1.0 - t)), c1 = (float)(gp * t);
            float c2 = (float)(gm * (1.0 - t)), c3 = (float)(gm * t);
            // lanes sit on different segments: reduce once per distinct segment
            uint64_t pend = __ballot(c0 != 0.0f || c1 != 0.0f || c2 != 0.0f || c3 != 0.0f);
            while (pend) {
                const int src = __ffsll((unsigned long long)pend) - 1;
                const int j0 = __shfl(j, src, 64);
                const bool mine = (j == j0);
                const float s0 = wave_sum(mine ? c0 : 0.0f), s1 = wave_sum(mine ? c1 : 0.0f);
                const float s2 = wave_sum(mine ? c2 : 0.0f), s3 = wave_sum(mine ? c3 : 0.0f);
                if ((threadIdx.x & 63) == 0) {
                    add_field(P, pr.f0 + 2 + j0, s0);
                    add_field(P, pr.f0 + 3 + j0, s1);
                    add_field(P, pr.f0 + 2 + M + j0, s2);
                    add_field(P, pr.f0 + 3 + M + j0, s3);
                }
                pend &= ~__ballot(mine);
            }
            break;
        }
    }
}

// ------------------------------------------------------------------ column kernel
template <int MODE, int NC, int TYPES, int SIGS>
__global__ __launch_bounds__(256) void k_column(const KParams P) {
    __shared__ int s_cand[kCandCap];
    __shared__ int s_cnt[kBlock / 64];
    const int tid = threadIdx.x, wave = tid >> 6;

    int b = blockIdx.x;
    const int seg = b % P.nseg;
    b /= P.nseg;
    const int tvi = b % P.tiles_v;
    b /= P.tiles_v;
    const int tui = b % P.tiles_u;
    const int comp = b / P.tiles_u;

    const int TU = P.tu;
    const int lu = tid & (TU - 1), lv = tid / TU;
    const int u = tui * TU + lu, v = tvi * P.tv + lv;
    const bool act = (u < P.nu) && (v < P.nv);
    const int uu = min(u, P.nu - 1), vv = min(v, P.nv - 1);
    const double* __restrict__ ucs = P.uc[comp];
    const double* __restrict__ vcs = P.vc[comp];
    const double uc = ucs[uu], uw = P.uw[comp][uu];
    const double vc = vcs[vv], vw = P.vw[comp][vv];

    Tile T;
    {
        const int u0 = tui * TU, u1 = min(u0 + TU, P.nu) - 1;
        const int v0 = tvi * P.tv, v1 = min(v0 + P.tv, P.nv) - 1;
        T.ulo = ucs[u0];
        T.uhi = ucs[u1];
        T.vlo = vcs[v0];
        T.vhi = vcs[v1];
        int wu0, wu1, wv0, wv1;
        if (TU <= 64) {
            wu0 = u0;
            wu1 = u1;
            wv0 = v0 + wave * (64 / TU);
            wv1 = min(wv0 + 64 / TU, P.nv) - 1;
        } else {
            wu0 = u0 + (wave * 64) % TU;
            wu1 = min(wu0 + 64, P.nu) - 1;
            wv0 = wv1 = v0 + (wave * 64) / TU;
        }
        T.wave_live = (wu0 < P.nu) && (wv0 < P.nv);
        T.wulo = ucs[min(wu0, P.nu - 1)];
        T.wuhi = ucs[max(0, min(wu1, P.nu - 1))];
        T.wvlo = vcs[min(wv0, P.nv - 1)];
        T.wvhi = vcs[max(0, min(wv1, P.nv - 1))];
    }

    double F[NC];
    int nlist;
    bool complete;
    inplane_sums<NC, TYPES, SIGS>(P, P.bbox, P.fval, T, uc, uw, vc, vw, s_cand, s_cnt, F, nlist, complete);
    double F2[NC];
    if constexpr (MODE == MODE_FD) {
        int nl2;
        bool c2;
        __syncthreads();
        inplane_sums<NC, TYPES, SIGS>(P, P.bbox2, P.fval2, T, uc, uw, vc, vw, s_cand, s_cnt, F2, nl2, c2);
    }

    const int w0 = seg * P.seglen;
    const int w1 = min(w0 + P.seglen, P.nw);
    const int64_t b0 = (int64_t)uu + (int64_t)vv * P.sv;     // offset within a component plane
    const double* __restrict__ zt0 = P.ztab + (int64_t)comp * P.nclass * P.nw * 3;

    float A[NC], Blo[NC], Bhi[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) A[c] = Blo[c] = Bhi[c] = 0.0f;

    if constexpr (MODE == MODE_EPS || MODE == MODE_FD) {
        const double* __restrict__ zt2 = (MODE == MODE_FD) ? P.ztab2 + (int64_t)comp * P.nclass * P.nw * 3 : nullptr;
        float* __restrict__ outp = P.out + (int64_t)comp * P.plane + b0;
#pragma unroll 2
        for (int w = w0; w < w1; ++w) {
            double Z[NC];
            const double s = compose<NC>(P, F, zt0 + 3 * w, Z).s;
            float out;
            if constexpr (MODE == MODE_EPS) {
                out = (float)(P.eps_bg + P.deps * s);
            } else {
                const double s2 = compose<NC>(P, F2, zt2 + 3 * w, Z).s;
                out = (float)(P.deps * (s - s2));
            }
            if (act) outp[(int64_t)w * P.sw] = out;
        }
        return;
    } else {
        const float2* __restrict__ efp = P.ef[comp];
        const float2* __restrict__ eap = P.ea[comp];
        const float* __restrict__ gpl = P.geps + (int64_t)comp * P.plane;
        // U column steps per iteration: every load of the group is issued before
        // the first one is used, so each wavefront keeps 2U loads in flight.
        constexpr int U = 4;
        for (int w = w0; w < w1; w += U) {
            float gs[U];
#pragma unroll
            for (int q = 0; q < U; ++q) {
                const int wq = min(w + q, w1 - 1);
                const int64_t i = b0 + (int64_t)wq * P.sw;
                if constexpr (MODE == MODE_VJP_FIELDS) {
                    const float2 e = efp[i], a = eap[i];
                    gs[q] = P.two_omega * (e.x * a.y + e.y * a.x);   // 2 omega Im(E Eadj)
                } else {
                    gs[q] = gpl[i];
                }
                if (!act || w + q >= w1) gs[q] = 0.0f;
            }
#pragma unroll
            for (int q = 0; q < U; ++q) {
                if (w + q < w1) {
                    double Z[NC];
                    const Comp o = compose<NC>(P, F, zt0 + 3 * (w + q), Z);
                    const float gd = gs[q] * (float)P.deps;
                    const float cg0 = gd * (float)o.r0, cg1 = gd * (float)o.r1;
                    const float cg2 = gd * (float)o.r2, cg3 = gd * (float)o.r3;
#pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        if (c < P.nclass) {
                            const int g = P.cls_group[c];
                            const float cc = (g == 0) ? cg0 : (g == 1) ? cg1 : (g == 2) ? cg2 : cg3;
                            A[c] += cc * (float)Z[c];
                            if (P.cls_wparam[c]) {
                                const double* z = zt0 + 3 * ((int64_t)c * P.nw + w + q);
                                Blo[c] += cc * (float)z[1];
                                Bhi[c] += cc * (float)z[2];
                            }
                        }
                    }
                }
            }
        }
    }

    // ---- end of the column: partials of the column-axis bounds of each class
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        if (c < P.nclass && P.cls_wparam[c] && T.wave_live) {
            const DevClass cl = P.cls[c];
            const float fs = act ? (float)F[c] : 0.0f;
            emit(P, cl.flo, fs * Blo[c]);
            emit(P, cl.fhi, fs * Bhi[c]);
        }
    }
    // ---- in-plane partials of every candidate
    if (!act) {
#pragma unroll
        for (int c = 0; c < NC; ++c) A[c] = 0.0f;
    }
    int next = 0;
    bool first = true;
    while (first || next < P.nprim) {
        int n;
        if (first && complete) {
            n = nlist;
            next = P.nprim;
        } else {
            __syncthreads();
            n = build_list(P.bbox, P.nprim, next, T.ulo, T.uhi, T.vlo, T.vhi, s_cand, s_cnt, &next);
        }
        first = false;
        if (!T.wave_live) continue;
        for (int j = 0; j < n; ++j) {
            const int pi = uniform_int(s_cand[j]);
            if (!wave_meets(T, P.bbox[pi])) continue;
            const DevPrim pr = P.prims[pi];
            const float a = class_pick<NC>(A, pr.cls);
            if (__ballot(a != 0.0f) == 0) continue;
            emit_partials<TYPES, SIGS>(P, pr, pi, a, uc, uw, vc, vw);
        }
    }
}

// ------------------------------------------------------------------ FD helpers
__global__ __launch_bounds__(256) void k_gplane(const float2* __restrict__ e0, const float2* __restrict__ e1,
                                                const float2* __restrict__ e2, const float2* __restrict__ a0,
                                                const float2* __restrict__ a1, const float2* __restrict__ a2,
                                                int ncomp, int64_t plane, float two_omega, float* __restrict__ g) {
    const int64_t n = (int64_t)ncomp * plane;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i / plane);
        const int64_t j = i - (int64_t)c * plane;
        const float2* e = c == 0 ? e0 : (c == 1 ? e1 : e2);
        const float2* a = c == 0 ? a0 : (c == 1 ? a1 : a2);
        const float2 ev = e[j], av = a[j];
        g[i] = two_omega * (ev.x * av.y + ev.y * av.x);
    }
}

__global__ __launch_bounds__(256) void k_dot(const float* __restrict__ a, const float* __restrict__ b, int64_t n,
                                             double scale, double* __restrict__ out) {
    __shared__ float red[4];
    float acc = 0.0f;
    const int64_t n4 = n / 4;
    const float4* a4 = reinterpret_cast<const float4*>(a);
    const float4* b4 = reinterpret_cast<const float4*>(b);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (int64_t)gridDim.x * blockDim.x) {
        const float4 x = a4[i], y = b4[i];
        acc += x.x * y.x + x.y * y.y + x.z * y.z + x.w * y.w;
    }
    for (int64_t i = 4 * n4 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        acc += a[i] * b[i];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        const float s = red[0] + red[1] + red[2] + red[3];
        if (s != 0.0f) atomicAdd(out, scale * (double)s);
    }
}

__global__ __launch_bounds__(256) void k_copy(uint4* __restrict__ dst, const uint4* __restrict__ src, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

__global__ __launch_bounds__(256) void k_fill(double* __restrict__ dst, double v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = v;
}

// ------------------------------------------------------------------ launchers
hipError_t launch_stage(const StageParams& sp, int nvariant, hipStream_t st) {
    const int64_t nz = (int64_t)sp.ncomp * sp.nclass * sp.nw;
    int64_t n = sp.nprim;
    if (nz > n) n = nz;
    if (sp.zero_n > n) n = sp.zero_n;
    if (n < 1) n = 1;
    const dim3 grid((unsigned)((n + 255) / 256), (unsigned)nvariant);
    hipLaunchKernelGGL(k_stage, grid, dim3(256), 0, st, sp);
    return hipGetLastError();
}

template <int MODE, int TYPES, int SIGS>
static hipError_t launch_variant(int ncls, const KParams& kp, hipStream_t st) {
    const int64_t blocks = (int64_t)kp.ncomp * kp.tiles_u * kp.tiles_v * kp.nseg;
    const dim3 grid((unsigned)blocks), blk(256);
    switch (ncls) {
        case 1: hipLaunchKernelGGL((k_column<MODE, 1, TYPES, SIGS>), grid, blk, 0, st, kp); break;
        case 2: hipLaunchKernelGGL((k_column<MODE, 2, TYPES, SIGS>), grid, blk, 0, st, kp); break;
        case 4: hipLaunchKernelGGL((k_column<MODE, 4, TYPES, SIGS>), grid, blk, 0, st, kp); break;
        default: hipLaunchKernelGGL((k_column<MODE, 8, TYPES, SIGS>), grid, blk, 0, st, kp); break;
    }
    return hipGetLastError();
}

template <int MODE>
static hipError_t launch_mode(int ncls, int variant, const KParams& kp, hipStream_t st) {
    switch (variant) {
        case VAR_BOX_LIN: return launch_variant<MODE, T_BOX, S_LIN>(ncls, kp, st);
        case VAR_GCART_LIN: return launch_variant<MODE, T_BOX | T_GCART, S_LIN>(ncls, kp, st);
        case VAR_ELL_SIGMOID: return launch_variant<MODE, T_BOX | T_ELL, S_LIN | S_SIGMOID>(ncls, kp, st);
        default: return launch_variant<MODE, T_ALL, S_ALL>(ncls, kp, st);
    }
}

hipError_t launch_column(int mode, int ncls, int variant, const KParams& kp, hipStream_t st) {
    switch (mode) {
        case MODE_EPS: return launch_mode<MODE_EPS>(ncls, variant, kp, st);
        case MODE_VJP_FIELDS: return launch_mode<MODE_VJP_FIELDS>(ncls, variant, kp, st);
        case MODE_VJP_GEPS: return launch_mode<MODE_VJP_GEPS>(ncls, variant, kp, st);
        default: return launch_mode<MODE_FD>(ncls, variant, kp, st);
    }
}

hipError_t launch_gplane(const float2* const* ef, const float2* const* ea, int ncomp, int64_t plane,
                         float two_omega, float* g, hipStream_t st) {
    const float2* e[3] = {ef[0], ncomp > 1 ? ef[1] : ef[0], ncomp > 2 ? ef[2] : ef[0]};
    const float2* a[3] = {ea[0], ncomp > 1 ? ea[1] : ea[0], ncomp > 2 ? ea[2] : ea[0]};
    hipLaunchKernelGGL(k_gplane, dim3(2048), dim3(256), 0, st, e[0], e[1], e[2], a[0], a[1], a[2], ncomp, plane,
                       two_omega, g);
    return hipGetLastError();
}

hipError_t launch_dot(const float* a, const float* b, int64_t n, double scale, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_dot, dim3(2048), dim3(256), 0, st, a, b, n, scale, out);
    return hipGetLastError();
}

hipError_t launch_copy(void* dst, const void* src, int64_t bytes, hipStream_t st) {
    hipLaunchKernelGGL(k_copy, dim3(4096), dim3(256), 0, st, (uint4*)dst, (const uint4*)src, bytes / 16);
    return hipGetLastError();
}

hipError_t launch_fill(double* dst, double v, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_fill, dim3((unsigned)std::min<int64_t>(1024, (n + 255) / 256 + 1)), dim3(256), 0, st, dst,
                       v, n);
    return hipGetLastError();
}

}  // namespace sg

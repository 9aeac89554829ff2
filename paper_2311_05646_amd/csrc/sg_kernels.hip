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
// Sum over the 64 lanes of a wavefront with DPP lane moves (no LDS traffic):
// quad swaps, row rotations, then the two row broadcasts of wave64; lane 63
// ends up with the total, which is returned to every lane.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_add(float v) {
    const int moved = __builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xF, false);
    return v + __int_as_float(moved);
}
__device__ __forceinline__ float wave_sum(float v) {
    v = dpp_add<0xB1, 0xF>(v);    // quad_perm [1,0,3,2]
    v = dpp_add<0x4E, 0xF>(v);    // quad_perm [2,3,0,1]
    v = dpp_add<0x124, 0xF>(v);   // row_ror:4
    v = dpp_add<0x128, 0xF>(v);   // row_ror:8
    v = dpp_add<0x142, 0xA>(v);   // row_bcast:15 -> rows 1, 3
    v = dpp_add<0x143, 0xC>(v);   // row_bcast:31 -> rows 2, 3
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
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

// zs points at the class-0 entry of this column step; class c sits zstride further.
template <int TREE>
__device__ __forceinline__ Comp compose(const KParams& P, const double (&F)[tree_nc(TREE)], const double* zs,
                                        int zstride, double (&Z)[tree_nc(TREE)]) {
    constexpr int NC = tree_nc(TREE);
    Comp o;
    if constexpr (TREE == TR_U1 || TREE == TR_U2) {
        double S = 0.0;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            Z[c] = zs[c * zstride];
            S += F[c] * Z[c];
        }
        o.s = fmin(1.0, S);
        o.r0 = S < 1.0 ? 1.0 : 0.0;
        o.r1 = o.r2 = o.r3 = 0.0;
        return o;
    } else if constexpr (TREE == TR_D11 || TREE == TR_D12) {
        Z[0] = zs[0];
        const double S0 = F[0] * Z[0];
        double S1 = 0.0;
#pragma unroll
        for (int c = 1; c < NC; ++c) {
            Z[c] = zs[c * zstride];
            S1 += F[c] * Z[c];
        }
        const double v0 = fmin(1.0, S0), v1 = fmin(1.0, S1);
        const double d = v0 - v1;
        o.s = fmax(0.0, d);
        const bool pass = d > 0.0;
        o.r0 = (pass && S0 < 1.0) ? 1.0 : 0.0;
        o.r1 = (pass && S1 < 1.0) ? -1.0 : 0.0;
        o.r2 = o.r3 = 0.0;
        return o;
    } else {
        double S0 = 0.0, S1 = 0.0, S2 = 0.0, S3 = 0.0;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if (c < P.nclass) {
                Z[c] = zs[c * zstride];
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
}


// Partials of a convex polygon at one sample, times a; one reduction per
// vertex field and edge.
template <int SIGS>
__device__ void poly_partials(const KParams& P, const DevPrim& pr, double ad, double uc, double vc) {
    const double* fv = P.fval;
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
}

// Partials of a two-sided piecewise-linear boundary, times the column sums,
// over the kBlock samples of the tile handled by this wavefront.  Each sample
// touches the y+ and y- of its segment's two vertices; the contributions are
// bucketed per vertex in this wavefront's LDS slice (ds_add_f32) and flushed
// with one atomic per touched vertex field.  Tiles that span more than
// kSegBucket vertices fall back to one reduction per distinct segment.
constexpr int kSegBucket = 256;

template <int SIGS>
__device__ void gcart_partials(const KParams& P, const DevPrim& pr, const float* sAc, int u0, int v0, int comp,
                               const Tile& T, float* sg) {
    constexpr int Q = kBlock / 64;
    const int lane = threadIdx.x & 63;
    const int TU = P.tu;
    const double* fv = P.fval;
    const int M = pr.nvert;
    const double* xv = P.consts + pr.c0;
    const double* yp = fv + pr.f0 + 2;
    const double* ym = yp + M;
    int jlo, jhi;
    double tdum;
    gcart_segment(xv, M, T.ulo, jlo, tdum);
    gcart_segment(xv, M, T.uhi, jhi, tdum);
    const int nvx = jhi - jlo + 2;               // vertices jlo .. jhi + 1
    const bool bucket = nvx <= kSegBucket;
    if (bucket) {
        for (int i = lane; i < 2 * nvx; i += 64) sg[i] = 0.0f;
        __builtin_amdgcn_s_waitcnt(0xc07f);      // lgkmcnt(0): the zeros are in LDS
        __builtin_amdgcn_wave_barrier();
    }
    double sxs = 0.0, sxe = 0.0;
#pragma unroll 1
    for (int q = 0; q < Q; ++q) {
        const int t = q * 64 + lane;
        const float a = sAc[t];
        if (__ballot(a != 0.0f) == 0) continue;
        const int uq = min(u0 + (t & (TU - 1)), P.nu - 1), vq = min(v0 + t / TU, P.nv - 1);
        const double uc = P.uc[comp][uq], uw = P.uw[comp][uq], vc = P.vc[comp][vq], vw = P.vw[comp][vq];
        const double ad = (double)a;
        float c0 = 0.0f, c1 = 0.0f, c2 = 0.0f, c3 = 0.0f;
        int j = 0;
        if (a != 0.0f) {
            double rx, drx0, drx1;
            rect_vd<SIGS>(pr.sk0, kval(pr.sm0, pr.k0, uw), uc, fv[pr.f0], fv[pr.f0 + 1], rx, drx0, drx1);
            double t01;
            gcart_segment(xv, M, uc, j, t01);
            const double fp = (1.0 - t01) * yp[j] + t01 * yp[j + 1];
            const double fm = (1.0 - t01) * ym[j] + t01 * ym[j + 1];
            const double ky = kval(pr.sm1, pr.k1, vw);
            double sp, dsp, sm, dsm;
            sig_vd<SIGS>(pr.sk1, ky * (fp - vc), sp, dsp);
            sig_vd<SIGS>(pr.sk1, ky * (vc - fm), sm, dsm);
            const double fy = sp * sm;
            sxs += ad * drx0 * fy;
            sxe += ad * drx1 * fy;
            const double gp = ad * rx * ky * dsp * sm;    // a * dF / d f+
            const double gm = -ad * rx * sp * ky * dsm;   // a * dF / d f-
            c0 = (float)(gp * (1.0 - t01));
            c1 = (float)(gp * t01);
            c2 = (float)(gm * (1.0 - t01));
            c3 = (float)(gm * t01);
        }
        if (bucket) {
            if (c0 != 0.0f || c1 != 0.0f || c2 != 0.0f || c3 != 0.0f) {
                const int k = j - jlo;
                atomicAdd(sg + k, c0);
                atomicAdd(sg + k + 1, c1);
                atomicAdd(sg + nvx + k, c2);
                atomicAdd(sg + nvx + k + 1, c3);
            }
        } else {
            uint64_t pend = __ballot(c0 != 0.0f || c1 != 0.0f || c2 != 0.0f || c3 != 0.0f);
            while (pend) {
                const int src = __ffsll((unsigned long long)pend) - 1;
                const int j0 = __shfl(j, src, 64);
                const bool mine = (j == j0);
                const float s0 = wave_sum(mine ? c0 : 0.0f), s1 = wave_sum(mine ? c1 : 0.0f);
                const float s2 = wave_sum(mine ? c2 : 0.0f), s3 = wave_sum(mine ? c3 : 0.0f);
                if (lane == 0) {
                    add_field(P, pr.f0 + 2 + j0, s0);
                    add_field(P, pr.f0 + 3 + j0, s1);
                    add_field(P, pr.f0 + 2 + M + j0, s2);
                    add_field(P, pr.f0 + 3 + M + j0, s3);
                }
                pend &= ~__ballot(mine);
            }
        }
    }
    emit(P, pr.f0, (float)sxs);
    emit(P, pr.f0 + 1, (float)sxe);
    if (bucket) {
        __builtin_amdgcn_s_waitcnt(0xc07f);
        __builtin_amdgcn_wave_barrier();
        for (int i = lane; i < 2 * nvx; i += 64) {
            const float v = sg[i];
            if (v != 0.0f) add_field(P, i < nvx ? pr.f0 + 2 + jlo + i : pr.f0 + 2 + M + jlo + (i - nvx), v);
        }
    }
}

// One candidate primitive, handled by one wavefront for all kBlock samples of
// the block's tile (kBlock / 64 samples per lane): in-plane partials times the
// class column sums sAc[sample], summed over the lane's samples, reduced over
// the wavefront, and added with one atomic per parameter field.
template <int TYPES, int SIGS>
__device__ void block_partials(const KParams& P, const DevPrim& pr, const float* sAc, int u0, int v0, int comp,
                               const Tile& T, float* sg) {
    constexpr int Q = kBlock / 64;
    const int lane = threadIdx.x & 63;
    const int TU = P.tu;
    const double* fv = P.fval;
    const int type = (TYPES == T_BOX) ? SG_PRIM_BOX : pr.type;
    if constexpr ((TYPES & T_BOX) != 0) {
        if (type == SG_PRIM_BOX) {
            double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll 1
            for (int q = 0; q < Q; ++q) {
                const int t = q * 64 + lane;
                const float a = sAc[t];
                if (a != 0.0f) {
                    const int uq = min(u0 + (t & (TU - 1)), P.nu - 1), vq = min(v0 + t / TU, P.nv - 1);
                    const double ad = (double)a;
                    double ru = 1.0, du0 = 0.0, du1 = 0.0, rv = 1.0, dv0 = 0.0, dv1 = 0.0;
                    if (pr.ubnd)
                        rect_vd<SIGS>(pr.sk0, kval(pr.sm0, pr.k0, P.uw[comp][uq]), P.uc[comp][uq], fv[pr.fu0],
                                      fv[pr.fu1], ru, du0, du1);
                    if (pr.vbnd)
                        rect_vd<SIGS>(pr.sk1, kval(pr.sm1, pr.k1, P.vw[comp][vq]), P.vc[comp][vq], fv[pr.fv0],
                                      fv[pr.fv1], rv, dv0, dv1);
                    s0 += ad * du0 * rv;
                    s1 += ad * du1 * rv;
                    s2 += ad * ru * dv0;
                    s3 += ad * ru * dv1;
                }
            }
            if (pr.ubnd) {
                emit(P, pr.fu0, (float)s0);
                emit(P, pr.fu1, (float)s1);
            }
            if (pr.vbnd) {
                emit(P, pr.fv0, (float)s2);
                emit(P, pr.fv1, (float)s3);
            }
            return;
        }
    }
    if constexpr ((TYPES & T_ELL) != 0) {
        if (type == SG_PRIM_ELLIPSE) {
            const double x0 = fv[pr.f0], y0 = fv[pr.f0 + 1], r = fv[pr.f0 + 2];
            const double rhi = r + pr.reach0, rlo = r - pr.reach0;
            double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll 1
            for (int q = 0; q < Q; ++q) {
                const int t = q * 64 + lane;
                const float a = sAc[t];
                if (a != 0.0f) {
                    const int uq = min(u0 + (t & (TU - 1)), P.nu - 1), vq = min(v0 + t / TU, P.nv - 1);
                    const double qx = (P.uc[comp][uq] - x0) * pr.iax, qy = (P.vc[comp][vq] - y0) * pr.iay;
                    const double rho2 = qx * qx + qy * qy;
                    if (rhi > 0.0 && rho2 < rhi * rhi && !(rlo > 0.0 && rho2 <= rlo * rlo)) {
                        // derivatives only: FP32 after the FP64 differences
                        const float fqx = (float)qx, fqy = (float)qy;
                        const float rho = sqrtf(fqx * fqx + fqy * fqy);
                        const float ds = sig_d32(pr.sk0, (float)pr.k0 * ((float)r - rho));
                        const float g = a * (float)pr.k0 * ds;     // a * dF / d(r - rho)
                        const float inv = rho > 0.0f ? 1.0f / rho : 0.0f;
                        s0 += (double)(g * fqx * inv * (float)pr.iax);   // -drho/dx0 = dx / (ax^2 rho)
                        s1 += (double)(g * fqy * inv * (float)pr.iay);
                        s2 += (double)g;
                    }
                }
            }
            emit(P, pr.f0, (float)s0);
            emit(P, pr.f0 + 1, (float)s1);
            emit(P, pr.f0 + 2, (float)s2);
            return;
        }
    }
    if constexpr ((TYPES & T_POLY) != 0) {
        if (type == SG_PRIM_POLY) {
#pragma unroll 1
            for (int q = 0; q < Q; ++q) {
                const int t = q * 64 + lane;
                const float a = sAc[t];
                if (__ballot(a != 0.0f) == 0) continue;
                const int uq = min(u0 + (t & (TU - 1)), P.nu - 1), vq = min(v0 + t / TU, P.nv - 1);
                poly_partials<SIGS>(P, pr, (double)a, P.uc[comp][uq], P.vc[comp][vq]);
            }
            return;
        }
    }
    if constexpr ((TYPES & T_GCART) != 0) {
        if (type == SG_PRIM_GCART) {
            gcart_partials<SIGS>(P, pr, sAc, u0, v0, comp, T, sg);
            return;
        }
    }
}

// ------------------------------------------------------------------ column kernel
template <int MODE, int TREE, int TYPES, int SIGS>
__device__ __forceinline__ void column_body(const KParams& P, int b) {
    constexpr int NC = tree_nc(TREE);
    __shared__ int s_cand[kCandCap];
    __shared__ int s_cnt[kBlock / 64];
    const int tid = threadIdx.x, wave = tid >> 6;

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

    // Column steps [w0, w1).  Field loads are double-buffered in two register
    // sets of U steps each: while one group is being composed the next one is
    // in flight.  The first group goes out before the in-plane pass.
    const int w0 = seg * P.seglen;
    const int w1 = min(w0 + P.seglen, P.nw);
    const int64_t b0 = (int64_t)uu + (int64_t)vv * P.sv;     // offset within a component plane
    constexpr bool VJP = (MODE == MODE_VJP_FIELDS || MODE == MODE_VJP_GEPS);
    constexpr int U = (MODE == MODE_VJP_GEPS) ? 8 : 4;
    const float2* __restrict__ efp = nullptr;
    const float2* __restrict__ eap = nullptr;
    const float* __restrict__ gep = nullptr;
    if constexpr (MODE == MODE_VJP_FIELDS) {
        efp = P.ef[comp] + b0;
        eap = P.ea[comp] + b0;
    } else if constexpr (MODE == MODE_VJP_GEPS) {
        gep = P.geps + (int64_t)comp * P.plane + b0;
    }
    struct Set {
        float2 e[U], a[U];
        float g[U];
    };
    Set sa, sb;
    auto load_set = [&](Set& st, int w) {
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int64_t off = (int64_t)min(w + q, w1 - 1) * P.sw;
            if constexpr (MODE == MODE_VJP_FIELDS) {
                st.e[q] = efp[off];
                st.a[q] = eap[off];
            } else if constexpr (MODE == MODE_VJP_GEPS) {
                st.g[q] = gep[off];
            }
        }
    };
    if constexpr (VJP) load_set(sa, w0);

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

    // LDS copy of the extrusion tables of this column range, CH steps at a time
    constexpr int NT = (MODE == MODE_FD) ? 2 : 1;
    constexpr int CH = ((kZStage / NT / NC) / (2 * U)) * (2 * U);
    __shared__ double sZ[NT * NC * CH];
    __shared__ float2 sZd[VJP ? NC * CH : 1];
    const int64_t zcomp = (int64_t)comp * P.nclass * P.nw * 3;
    auto stage_z = [&](int wc) {
        __syncthreads();
        const int len = min(CH, w1 - wc);
        const int tot = NT * P.nclass * len;
        for (int i = tid; i < tot; i += kBlock) {
            const int tb = i / (P.nclass * len), r = i - tb * (P.nclass * len);
            const int c = r / len, j = r - c * len;
            const double* z = (tb == 0 ? P.ztab : P.ztab2) + zcomp + 3 * ((int64_t)c * P.nw + wc + j);
            sZ[(tb * NC + c) * CH + j] = z[0];
            if constexpr (VJP) sZd[c * CH + j] = make_float2((float)z[1], (float)z[2]);
        }
        __syncthreads();
    };

    float A[NC], Blo[NC], Bhi[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) A[c] = Blo[c] = Bhi[c] = 0.0f;

    if constexpr (MODE == MODE_EPS || MODE == MODE_FD) {
        float* __restrict__ outp = P.out + (int64_t)comp * P.plane + b0;
        for (int wc = w0; wc < w1; wc += CH) {
            stage_z(wc);
            const int we = min(wc + CH, w1);
#pragma unroll 2
            for (int w = wc; w < we; ++w) {
                double Z[NC];
                const double s = compose<TREE>(P, F, sZ + (w - wc), CH, Z).s;
                float out;
                if constexpr (MODE == MODE_EPS) {
                    out = (float)(P.eps_bg + P.deps * s);
                } else {
                    const double s2 = compose<TREE>(P, F2, sZ + NC * CH + (w - wc), CH, Z).s;
                    out = (float)(P.deps * (s - s2));
                }
                if (act) outp[(int64_t)w * P.sw] = out;
            }
        }
        return;
    } else {
        int wc = w0;   // first step of the staged chunk
        auto process = [&](const Set& st, int w) {
            if ((w - w0) % CH == 0) {
                wc = w;
                stage_z(w);
            }
            float gs[U];
#pragma unroll
            for (int q = 0; q < U; ++q) {
                if constexpr (MODE == MODE_VJP_FIELDS)
                    gs[q] = P.two_omega * (st.e[q].x * st.a[q].y + st.e[q].y * st.a[q].x);   // 2 omega Im(E Eadj)
                else
                    gs[q] = st.g[q];
                if (!act || w + q >= w1) gs[q] = 0.0f;
            }
#pragma unroll
            for (int q = 0; q < U; ++q) {
                if (w + q < w1) {
                    const int j = w + q - wc;
                    double Z[NC];
                    const Comp o = compose<TREE>(P, F, sZ + j, CH, Z);
                    const float gd = gs[q] * (float)P.deps;
                    const float cg0 = gd * (float)o.r0, cg1 = gd * (float)o.r1;
                    const float cg2 = gd * (float)o.r2, cg3 = gd * (float)o.r3;
#pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        if (c < P.nclass) {
                            constexpr int fixed = tree_group(TREE, 0) >= 0;
                            const int g = fixed ? tree_group(TREE, c) : P.cls_group[c];
                            const float cc = (g == 0) ? cg0 : (g == 1) ? cg1 : (g == 2) ? cg2 : cg3;
                            A[c] += cc * (float)Z[c];
                            if (P.cls_wparam[c]) {
                                const float2 zd = sZd[c * CH + j];
                                Blo[c] += cc * zd.x;
                                Bhi[c] += cc * zd.y;
                            }
                        }
                    }
                }
            }
        };
        const int ngrp = (w1 - w0 + U - 1) / U;
        for (int gi = 0; gi < ngrp; gi += 2) {
            if (gi + 1 < ngrp) load_set(sb, w0 + (gi + 1) * U);
            process(sa, w0 + gi * U);
            if (gi + 1 < ngrp) {
                if (gi + 2 < ngrp) load_set(sa, w0 + (gi + 2) * U);
                process(sb, w0 + (gi + 1) * U);
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
    // ---- in-plane partials: column sums to LDS, candidates split over the
    // block's wavefronts, one atomic per (block, parameter field)
    __shared__ float sA[NC * kBlock];
    __shared__ float sG[(TYPES & T_GCART) ? (kBlock / 64) * 2 * kSegBucket : 1];
#pragma unroll
    for (int c = 0; c < NC; ++c) sA[c * kBlock + tid] = act ? A[c] : 0.0f;
    __syncthreads();
    const int u0 = tui * TU, v0 = tvi * P.tv;
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
        for (int j = wave; j < n; j += kBlock / 64) {
            const int pi = uniform_int(s_cand[j]);
            const DevPrim pr = P.prims[pi];
            block_partials<TYPES, SIGS>(P, pr, sA + pr.cls * kBlock, u0, v0, comp, T, sG + wave * 2 * kSegBucket);
        }
    }
}

template <int MODE, int TREE, int TYPES, int SIGS>
__global__ __launch_bounds__(256) void k_column(const KParams P) {
    column_body<MODE, TREE, TYPES, SIGS>(P, blockIdx.x);
}

// Several requests in one launch: request r owns blocks [first[r], first[r+1])
// and its own parameter block plist[r] (same kernel specialization).
template <int MODE, int TREE, int TYPES, int SIGS>
__global__ __launch_bounds__(256) void k_column_batch(const KParams* __restrict__ plist,
                                                      const int* __restrict__ first, int nreq) {
    int lo = 0, hi = nreq;                   // first[lo] <= blockIdx.x < first[hi]
    const int b = blockIdx.x;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (first[mid] <= b) lo = mid; else hi = mid;
    }
    column_body<MODE, TREE, TYPES, SIGS>(plist[lo], b - first[lo]);
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

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of two 32x32
// multiplies, key bumped by the Weyl constants between rounds.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Element i of E and Eadj: Philox of counter (i_lo, i_hi, 0, 0) under key
// (seed_lo, seed_hi); u_k = (x_k + 1/2) 2^-32; two Box-Muller pairs give
// (Re E, Im E) from (u0, u1) and (Re Eadj, Im Eadj) from (u2, u3).
__global__ __launch_bounds__(256) void k_fieldgen(float2* __restrict__ e, float2* __restrict__ a, int64_t n,
                                                  uint32_t k0, uint32_t k1) {
    const float scale = 2.3283064365386963e-10f;   // 2^-32
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint4 x = philox4x32_10(make_uint4((uint32_t)i, (uint32_t)(i >> 32), 0u, 0u), k0, k1);
        const float u0 = ((float)x.x + 0.5f) * scale, u1 = ((float)x.y + 0.5f) * scale;
        const float u2 = ((float)x.z + 0.5f) * scale, u3 = ((float)x.w + 0.5f) * scale;
        const float r0 = sqrtf(-2.0f * logf(u0)), r1 = sqrtf(-2.0f * logf(u2));
        float s0, c0, s1, c1;
        sincosf(6.283185307179586f * u1, &s0, &c0);
        sincosf(6.283185307179586f * u3, &s1, &c1);
        e[i] = make_float2(r0 * c0, r0 * s0);
        a[i] = make_float2(r1 * c1, r1 * s1);
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
static hipError_t launch_variant(int tree, const KParams& kp, hipStream_t st) {
    const int64_t blocks = (int64_t)kp.ncomp * kp.tiles_u * kp.tiles_v * kp.nseg;
    const dim3 grid((unsigned)blocks), blk(256);
    switch (tree) {
        case TR_U1: hipLaunchKernelGGL((k_column<MODE, TR_U1, TYPES, SIGS>), grid, blk, 0, st, kp); break;
        case TR_U2: hipLaunchKernelGGL((k_column<MODE, TR_U2, TYPES, SIGS>), grid, blk, 0, st, kp); break;
        case TR_D11: hipLaunchKernelGGL((k_column<MODE, TR_D11, TYPES, SIGS>), grid, blk, 0, st, kp); break;
        case TR_D12: hipLaunchKernelGGL((k_column<MODE, TR_D12, TYPES, SIGS>), grid, blk, 0, st, kp); break;
        default:
            // generic op trees only come with the catch-all feature set
            if constexpr (TYPES == T_ALL && SIGS == S_ALL) {
                if (tree == TR_GEN4) hipLaunchKernelGGL((k_column<MODE, TR_GEN4, TYPES, SIGS>), grid, blk, 0, st, kp);
                else hipLaunchKernelGGL((k_column<MODE, TR_GEN8, TYPES, SIGS>), grid, blk, 0, st, kp);
            } else {
                return hipErrorInvalidValue;
            }
            break;
    }
    return hipGetLastError();
}

template <int MODE, int TYPES, int SIGS>
static hipError_t launch_batch_variant(int tree, const KParams* plist, const int* first, int nreq, int64_t blocks,
                                       hipStream_t st) {
    const dim3 grid((unsigned)blocks), blk(256);
    switch (tree) {
        case TR_U1: hipLaunchKernelGGL((k_column_batch<MODE, TR_U1, TYPES, SIGS>), grid, blk, 0, st, plist, first, nreq); break;
        case TR_U2: hipLaunchKernelGGL((k_column_batch<MODE, TR_U2, TYPES, SIGS>), grid, blk, 0, st, plist, first, nreq); break;
        case TR_D11: hipLaunchKernelGGL((k_column_batch<MODE, TR_D11, TYPES, SIGS>), grid, blk, 0, st, plist, first, nreq); break;
        case TR_D12: hipLaunchKernelGGL((k_column_batch<MODE, TR_D12, TYPES, SIGS>), grid, blk, 0, st, plist, first, nreq); break;
        default:
            if constexpr (TYPES == T_ALL && SIGS == S_ALL) {
                if (tree == TR_GEN4)
                    hipLaunchKernelGGL((k_column_batch<MODE, TR_GEN4, TYPES, SIGS>), grid, blk, 0, st, plist, first, nreq);
                else
                    hipLaunchKernelGGL((k_column_batch<MODE, TR_GEN8, TYPES, SIGS>), grid, blk, 0, st, plist, first, nreq);
            } else {
                return hipErrorInvalidValue;
            }
            break;
    }
    return hipGetLastError();
}

hipError_t launch_column_batch(int tree, int variant, const KParams* plist, const int* first, int nreq,
                               int64_t blocks, hipStream_t st) {
    switch (variant) {
        case VAR_BOX_LIN: return launch_batch_variant<MODE_VJP_FIELDS, T_BOX, S_LIN>(tree, plist, first, nreq, blocks, st);
        case VAR_GCART_LIN:
            return launch_batch_variant<MODE_VJP_FIELDS, T_BOX | T_GCART, S_LIN>(tree, plist, first, nreq, blocks, st);
        case VAR_ELL_SIGMOID:
            return launch_batch_variant<MODE_VJP_FIELDS, T_BOX | T_ELL, S_LIN | S_SIGMOID>(tree, plist, first, nreq, blocks,
                                                                                          st);
        default: return launch_batch_variant<MODE_VJP_FIELDS, T_ALL, S_ALL>(tree, plist, first, nreq, blocks, st);
    }
}

template <int MODE>
static hipError_t launch_mode(int tree, int variant, const KParams& kp, hipStream_t st) {
    switch (variant) {
        case VAR_BOX_LIN: return launch_variant<MODE, T_BOX, S_LIN>(tree, kp, st);
        case VAR_GCART_LIN: return launch_variant<MODE, T_BOX | T_GCART, S_LIN>(tree, kp, st);
        case VAR_ELL_SIGMOID: return launch_variant<MODE, T_BOX | T_ELL, S_LIN | S_SIGMOID>(tree, kp, st);
        default: return launch_variant<MODE, T_ALL, S_ALL>(tree, kp, st);
    }
}

hipError_t launch_column(int mode, int tree, int variant, const KParams& kp, hipStream_t st) {
    switch (mode) {
        case MODE_EPS: return launch_mode<MODE_EPS>(tree, variant, kp, st);
        case MODE_VJP_FIELDS: return launch_mode<MODE_VJP_FIELDS>(tree, variant, kp, st);
        case MODE_VJP_GEPS: return launch_mode<MODE_VJP_GEPS>(tree, variant, kp, st);
        default: return launch_mode<MODE_FD>(tree, variant, kp, st);
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

hipError_t launch_fieldgen(float2* e, float2* a, int64_t n, uint64_t seed, hipStream_t st) {
    const int64_t blocks = std::min<int64_t>(8192, (n + 255) / 256);
    hipLaunchKernelGGL(k_fieldgen, dim3((unsigned)std::max<int64_t>(1, blocks)), dim3(256), 0, st, e, a, n,
                       (uint32_t)seed, (uint32_t)(seed >> 32));
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

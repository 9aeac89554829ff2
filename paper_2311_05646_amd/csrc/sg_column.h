// Column kernel of the shape-gradient path (templates), included by the
// translation units that instantiate its modes (sg_mode_*.hip) and by
// sg_kernels.hip (launch dispatch).
//
//  k_column  one thread per in-plane sample (u, v) of one component, walking
//            a segment of its column (w).  In-plane factors F_h of the
//            candidate primitives are summed per extrusion class once per
//            column in FP64; along the column the composition (eq:union,
//            eq:intersection, difference) is evaluated once per run of steps
//            with equal extrusion masks, and either eps is stored (MODE_EPS),
//            the FD difference plane is stored (MODE_FD), or the reverse-mode
//            column sums A_c = sum_w g * d eps / d s_c * Z_c(w) are accumulated
//            (MODE_VJP_*) with g = 2 omega Im(E Eadj) (eq:1) or an upstream
//            dF/deps.  After the column the in-plane partials are multiplied
//            by A_c and reduced across the wavefront; lane 0 adds one FP64
//            atomic per parameter field touched by the wavefront.
#pragma once

#include <hip/hip_ext.h>

#include "sg_device.h"

namespace sg {

// ------------------------------------------------------------------ helpers
// Sum over the 64 lanes of a wavefront with DPP lane moves (no LDS traffic):
// quad swaps, row rotations, then the two row broadcasts of wave64; lane 63
// ends up with the total, which is returned to every lane.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_add(float v) {
    const int moved = __builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xF, false);
    return v + __int_as_float(moved);
}
// One exchange stage of a reduce-scatter over a 16-lane row: a[0 .. 2H) hold
// the lane's values for 2H terms; the lane keeps the half its H bit selects,
// adds the partner's values for that half (the partner, reached by the DPP
// control CTRL, has the other H bit) and leaves them in a[0 .. H).
template <int H, int CTRL>
__device__ __forceinline__ void row_scatter_sum(float (&a)[16], int lane) {
    const bool hi = (lane & H) != 0;
#pragma unroll
    for (int j = 0; j < H; ++j) {
        const float keep = hi ? a[H + j] : a[j];
        const float send = hi ? a[j] : a[H + j];
        a[j] = keep + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(send), CTRL, 0xF, 0xF, false));
    }
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

// Adds v to the fixed-point accumulators acc[0 .. 2] of one parameter.  v is
// rounded down to a multiple of 2^-64 and split into its integer part
// (|.| <= 2^31) and the two 32-bit halves of its 64 fraction bits; each piece
// goes into its own 64-bit integer accumulator, which fewer than 2^31 such
// additions cannot overflow.  Integer addition is associative, so the three
// sums, and the value k_fx_finish rebuilds from them, do not depend on the
// order in which the additions arrive.  |v| >= 2^31 or NaN sets *flag.
__device__ __forceinline__ void fx_add(unsigned long long* acc, unsigned long long* flag, double v) {
    if (!(fabs(v) < 0x1p31)) {
        atomicOr(flag, 1ull);
        return;
    }
    const double fl = floor(v);
    const unsigned long long f = (unsigned long long)((v - fl) * 0x1p64);   // v - fl is exact, in [0, 1)
    atomicAdd(acc, f & 0xffffffffull);
    atomicAdd(acc + 1, f >> 32);
    atomicAdd(acc + 2, (unsigned long long)(long long)fl);                  // two's complement
}

// The block's copy of the gradient (one of kGradSpread when P.gstride != 0).
__device__ __forceinline__ double* grad_copy(const KParams& P) {
    return P.grad + (int64_t)(blockIdx.x & (kGradSpread - 1)) * P.gstride;
}

// Adds v to grad[idx]: an FP64 atomic into the block's copy, or in
// deterministic mode the order-independent fixed-point sum.
__device__ __forceinline__ void grad_add(const KParams& P, int idx, double v) {
    if (P.fx) fx_add(P.fx + 3 * (int64_t)idx, P.fx + 3 * P.fx_n, v);
    else atomicAdd(grad_copy(P) + idx, v);
}

// Adds the wavefront sum of v (one value per lane) times the field's scale b
// to grad[idx] (idx < 0: a constant field).  Called with wave-uniform control flow.
__device__ __forceinline__ void emit_ref(const KParams& P, int idx, double b, float v) {
    if (idx < 0) return;
    if (__ballot(v != 0.0f) == 0) return;
    const float s = wave_sum(v);
    if ((threadIdx.x & 63) == 0) grad_add(P, idx, b * (double)s);
}
__device__ __forceinline__ void emit(const KParams& P, int field, float v) {
    const sg_field r = P.fref[field];
    emit_ref(P, r.idx, r.b, v);
}

// Field references [base, base + 64) of a primitive (those below `end`), one
// per lane, loaded together: a run of emits then waits for one memory round
// trip instead of one per emit (each emit branches on its field's index).
struct FieldWin {
    int base, idx;
    double b;
};
__device__ __forceinline__ void load_win(const KParams& P, FieldWin& w, int base, int end) {
    const int l = threadIdx.x & 63;
    w.base = base;
    w.idx = -1;
    w.b = 0.0;
    if (base + l < end) {
        const sg_field r = P.fref[base + l];
        w.idx = (int)r.idx;
        w.b = r.b;
    }
}
// The index and scale of field `field` (wave-uniform, base <= field < base + 64).
__device__ __forceinline__ void win_ref(const FieldWin& w, int field, int& idx, double& b) {
    const int l = uniform_int(field - w.base);
    idx = __builtin_amdgcn_readlane(w.idx, l);
    const long long bits = __double_as_longlong(w.b);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(bits & 0xffffffffll), l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)((unsigned long long)bits >> 32), l);
    b = __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ void emit_win(const KParams& P, const FieldWin& w, int field, float v) {
    int idx;
    double b;
    win_ref(w, field, idx, b);
    emit_ref(P, idx, b, v);
}

// One thread's v for a field (deterministic mode: one thread of the wavefront
// at a time, see gcart_partials).
__device__ __forceinline__ void add_field(const KParams& P, int field, float v) {
    const sg_field r = P.fref[field];
    if (r.idx >= 0 && v != 0.0f) grad_add(P, (int)r.idx, r.b * (double)v);
}

// Appends (in primitive order) every primitive in [start, start + kScan)
// whose support box meets the tile [ulo, uhi] x [vlo, vhi] to s_cand.  The
// kScan / kBlock support boxes of a thread are loaded together, so a pass costs
// one memory round trip and two barriers.  Returns the count; *next = first
// primitive not scanned.
constexpr int kScanPer = kCandCap / kBlock;     // support boxes per thread and pass
constexpr int kScan = kScanPer * kBlock;        // primitives per pass (never overflows s_cand)
constexpr int kScanCnt = kScanPer * (kBlock / 64);   // s_cnt entries
__device__ int scan_candidates(const float4* __restrict__ bb, int nprim, int start, double ulo, double uhi,
                               double vlo, double vhi, int* s_cand, int* s_cnt, int* next) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    constexpr int NW = kBlock / 64;
    // only the rows of kBlock boxes that hold primitives are read
    const int rows = min(kScanPer, (nprim - start + kBlock - 1) / kBlock);
    float4 box[kScanPer];
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        const int i = start + k * kBlock + tid;
        if (k < rows) box[k] = bb[min(i, nprim - 1)];
    }
    uint64_t m[kScanPer];
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        const int i = start + k * kBlock + tid;
        bool hit = false;
        if (k < rows) {
            const float4 b = box[k];
            hit = (i < nprim) && ((double)b.x <= uhi) && ((double)b.y >= ulo) && ((double)b.z <= vhi) &&
                  ((double)b.w >= vlo);
        }
        m[k] = __ballot(hit);
        if (lane == 0) s_cnt[k * NW + wave] = __popcll(m[k]);
    }
    __syncthreads();
    int off = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
#pragma unroll
        for (int q = 0; q < NW; ++q) {
            const int cq = s_cnt[k * NW + q];
            if (q < wave) off += cq;   // earlier wavefronts of this k
            tot += cq;
        }
        const int i = start + k * kBlock + tid;
        if ((m[k] >> lane) & 1ull) s_cand[off + __popcll(m[k] & ((1ull << lane) - 1ull))] = i;
        // the next k starts after every hit of this k
        for (int q = wave; q < NW; ++q) off += s_cnt[k * NW + q];
    }
    __syncthreads();
    *next = start + kScan;
    return tot;
}

struct Tile {
    double ulo, uhi, vlo, vhi;      // block: centers of the first / last sample
    double wulo, wuhi, wvlo, wvhi;  // this wavefront
    bool wave_live;
};

__device__ __forceinline__ bool wave_meets(const Tile& T, const double4& b) {
    return (b.x <= T.wuhi) && (b.y >= T.wulo) && (b.z <= T.wvhi) && (b.w >= T.wvlo);
}

template <int NC>
__device__ __forceinline__ void add_to_class(double (&F)[NC], int cls, double v) {
#pragma unroll
    for (int c = 0; c < NC; ++c)
        if (c == cls) F[c] += v;
}


// Copies the records of candidates s_cand[j0, j0 + n) (n <= kStageRec) to
// s_rec, one thread per candidate; barriers before (earlier readers) and after.
__device__ __forceinline__ void stage_cands(const PrimRec* __restrict__ prec, const int* s_cand, int j0, int n,
                                            PrimRec* s_rec) {
    __syncthreads();
    const int t = threadIdx.x;
    if (t < n) s_rec[t] = prec[s_cand[j0 + t]];
    __syncthreads();
}

// In-plane factor F(u, v) of a staged candidate (value only).
template <int TYPES, int SIGS>
__device__ __forceinline__ double cand_value(const KParams& P, const PrimRec& c, const double* __restrict__ fv,
                                             int comp, int u, double uc, double uw, double vc, double vw) {
    const DevPrim& pr = c.pr;
    if constexpr ((TYPES & T_BOX) != 0) {
        if (TYPES == T_BOX || pr.type == SG_PRIM_BOX) {
            double f = 1.0;
            if (pr.ubnd) f = rect_v<SIGS>(pr.sk0, kval(pr.sm0, pr.k0, uw), uc, c.f[0], c.f[1]);
            if (pr.vbnd) f *= rect_v<SIGS>(pr.sk1, kval(pr.sm1, pr.k1, vw), vc, c.f[2], c.f[3]);
            return f;
        }
    }
    if constexpr ((TYPES & T_ELL) != 0) {
        if (pr.type == SG_PRIM_ELLIPSE) {
            const double dx = (uc - c.f[0]) * pr.iax, dy = (vc - c.f[1]) * pr.iay;
            const double rho2 = dx * dx + dy * dy;
            const double r = c.f[2];
            const double rhi = r + pr.reach0, rlo = r - pr.reach0;
            if (rhi <= 0.0 || rho2 >= rhi * rhi) return 0.0;      // beyond the sigma support
            if (rlo > 0.0 && rho2 <= rlo * rlo) return 1.0;
            return sig_v<SIGS>(pr.sk0, pr.k0 * (r - sqrt(rho2)));
        }
    }
    if constexpr ((TYPES & (T_POLY | T_GCART | T_POLAR | T_SERIES)) != 0)
        return prim_value<TYPES & (T_POLY | T_GCART | T_POLAR | T_SERIES), SIGS>(pr, fv, P.consts, uc, uw, vc, vw,
                                                            P.gseg + pr.gs0 + (int64_t)comp * P.nu + u);
    return 0.0;
}

// cand_value, and in *live whether some in-plane partial of the candidate can
// be nonzero at the sample (see prim_value_live): for a box, a bound's sigma
// argument inside its support with the other axis' factor nonzero; for an
// ellipse, the sample inside the annulus where the partials code evaluates
// sigma' (widened by a relative 1e-9).
template <int TYPES, int SIGS>
__device__ __forceinline__ double cand_value_live(const KParams& P, const PrimRec& c, const double* __restrict__ fv,
                                                  int comp, int u, double uc, double uw, double vc, double vw,
                                                  bool& live) {
    const DevPrim& pr = c.pr;
    if constexpr ((TYPES & T_BOX) != 0) {
        if (TYPES == T_BOX || pr.type == SG_PRIM_BOX) {
            double ru = 1.0, rv = 1.0;
            bool lu = false, lv = false;
            if (pr.ubnd) {
                const double k = kval(pr.sm0, pr.k0, uw);
                const double ta = k * (uc - c.f[0]), tb = k * (c.f[1] - uc);
                ru = sig_v<SIGS>(pr.sk0, ta) * sig_v<SIGS>(pr.sk0, tb);
                lu = sig_live<SIGS>(pr.sk0, ta) || sig_live<SIGS>(pr.sk0, tb);
            }
            if (pr.vbnd) {
                const double k = kval(pr.sm1, pr.k1, vw);
                const double ta = k * (vc - c.f[2]), tb = k * (c.f[3] - vc);
                rv = sig_v<SIGS>(pr.sk1, ta) * sig_v<SIGS>(pr.sk1, tb);
                lv = sig_live<SIGS>(pr.sk1, ta) || sig_live<SIGS>(pr.sk1, tb);
            }
            live = (lu && rv != 0.0) || (lv && ru != 0.0);
            return ru * rv;
        }
    }
    if constexpr ((TYPES & T_ELL) != 0) {
        if (pr.type == SG_PRIM_ELLIPSE) {
            const double dx = (uc - c.f[0]) * pr.iax, dy = (vc - c.f[1]) * pr.iay;
            const double rho2 = dx * dx + dy * dy;
            const double r = c.f[2];
            const double rhi = r + pr.reach0, rlo = r - pr.reach0;
            live = rhi > 0.0 && rho2 < rhi * rhi * (1.0 + kSupportSlack) &&
                   !(rlo > 0.0 && rho2 <= rlo * rlo * (1.0 - kSupportSlack));
            if (rhi <= 0.0 || rho2 >= rhi * rhi) return 0.0;
            if (rlo > 0.0 && rho2 <= rlo * rlo) return 1.0;
            return sig_v<SIGS>(pr.sk0, pr.k0 * (r - sqrt(rho2)));
        }
    }
    if constexpr ((TYPES & (T_POLY | T_GCART | T_POLAR | T_SERIES)) != 0)
        return prim_value_live<TYPES & (T_POLY | T_GCART | T_POLAR | T_SERIES), SIGS>(pr, fv, P.consts, uc, uw, vc, vw,
                                                                 P.gseg + pr.gs0 + (int64_t)comp * P.nu + u, live);
    live = false;
    return 0.0;
}

// Sum of F_h over the candidates, per class, at (uc, vc).  When every
// candidate of the tile fits one staging round, the records stay in s_rec for
// the partials (*staged_all; *ncand of them).  after_stage() runs once, after
// the first staging round and before any evaluation (the caller issues its
// field loads there: vector loads return in order, so loads issued earlier
// would hold up the scan's and the staging's).  With PROBE, *live tells
// whether some candidate's in-plane partials can be nonzero at the sample.
template <int NC, int TYPES, int SIGS, bool PROBE = false, class Hook>
__device__ __forceinline__ void inplane_sums(const KParams& P, const float4* __restrict__ bbox,
                                             const PrimRec* __restrict__ prec, const double* __restrict__ fval,
                                             const Tile& T, int comp, int u, double uc, double uw, double vc,
                                             double vw, int* s_cand, int* s_cnt, PrimRec* s_rec, double (&F)[NC],
                                             int& ncand, bool& staged_all, Hook&& after_stage, bool* live = nullptr,
                                             bool eval = true) {
    // eval false: F is given (the F cache); only the candidates are listed and staged
    if (eval) {
#pragma unroll
        for (int c = 0; c < NC; ++c) F[c] = 0.0;
    }
    if constexpr (PROBE) *live = false;
    ncand = 0;
    staged_all = false;
    bool hooked = false;
    for (int next = 0; next < P.nprim;) {
        const bool first = next == 0;
        const int n = scan_candidates(bbox, P.nprim, next, T.ulo, T.uhi, T.vlo, T.vhi, s_cand, s_cnt, &next);
        if (first && next >= P.nprim && n <= kStageRec) {
            staged_all = true;
            ncand = n;
        }
        for (int j0 = 0; j0 < n; j0 += kStageRec) {
            const int nj = min(kStageRec, n - j0);
            stage_cands(prec, s_cand, j0, nj, s_rec);
            if (!hooked) {
                after_stage();
                hooked = true;
            }
            if (!T.wave_live || !eval) continue;
            for (int j = 0; j < nj; ++j) {
                if (!wave_meets(T, s_rec[j].bb)) continue;
                double f;
                if constexpr (PROBE) {
                    bool l;
                    f = cand_value_live<TYPES, SIGS>(P, s_rec[j], fval, comp, u, uc, uw, vc, vw, l);
                    *live = *live || l;
                } else {
                    f = cand_value<TYPES, SIGS>(P, s_rec[j], fval, comp, u, uc, uw, vc, vw);
                }
                add_to_class(F, s_rec[j].pr.cls, f);
            }
        }
    }
    if (!hooked) after_stage();
}

// Composition at one column step: root value s and, per class c, the
// derivative cf_c = d s / d (F_c Z_c) (0, +-1, or a product of the levels
// root's ratios).
template <int NC>
struct Comp {
    double s;
    double cf[NC];
};

// Extrusion factors of a step on which every class factor is exactly 0 or 1:
// bit c of mask set <=> Z_c = 1.
template <int NC>
__device__ __forceinline__ void mask_z(uint32_t mask, double (&Z)[NC]) {
#pragma unroll
    for (int c = 0; c < NC; ++c) Z[c] = ((mask >> c) & 1u) ? 1.0 : 0.0;
}

template <int TREE>
__device__ __forceinline__ Comp<tree_nc(TREE)> compose(const KParams& P, const double (&F)[tree_nc(TREE)],
                                                       const double (&Z)[tree_nc(TREE)]) {
    constexpr int NC = tree_nc(TREE);
    Comp<NC> o;
    if constexpr (TREE == TR_U1 || TREE == TR_U2) {
        double S = 0.0;
#pragma unroll
        for (int c = 0; c < NC; ++c) S += F[c] * Z[c];
        o.s = fmin(1.0, S);
        const double m = S < 1.0 ? 1.0 : 0.0;
#pragma unroll
        for (int c = 0; c < NC; ++c) o.cf[c] = m;
        return o;
    } else if constexpr (TREE == TR_D11 || TREE == TR_D12) {
        const double S0 = F[0] * Z[0];
        double S1 = 0.0;
#pragma unroll
        for (int c = 1; c < NC; ++c) S1 += F[c] * Z[c];
        const double v0 = fmin(1.0, S0), v1 = fmin(1.0, S1);
        const double d = v0 - v1;
        o.s = fmax(0.0, d);
        const bool pass = d > 0.0;
        o.cf[0] = (pass && S0 < 1.0) ? 1.0 : 0.0;
        const double r1 = (pass && S1 < 1.0) ? -1.0 : 0.0;
#pragma unroll
        for (int c = 1; c < NC; ++c) o.cf[c] = r1;
        return o;
    } else {
        // the general program: node sums in postfix order, then the chain
        // rule back from the root (every node has one parent, after it).
        // The clamp derivatives are bits of `passm`; a levels root keeps only
        // its children's values.
        constexpr int NN = kMaxNodes;
        double acc[NN], lvv[NN], r[NN];
#pragma unroll
        for (int k = 0; k < NN; ++k) acc[k] = lvv[k] = r[k] = 0.0;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if (c < P.nclass) {
                const double t = P.cls_sign[c] * (F[c] * Z[c]);
                const int kn = P.cls_node[c];
#pragma unroll
                for (int k = 0; k < NN; ++k)
                    if (kn == k) acc[k] += t;
            }
        }
        const int root = P.nnode - 1;
        const bool lev_root = P.node_op[root] == SG_OP_LEVELS;
        uint32_t passm = 0u;
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < NN; ++k) {
            if (k < P.nnode && !(lev_root && k == root)) {
                const int op = P.node_op[k];
                const double S = acc[k];
                double v;
                bool ps;
                if (op == SG_OP_UNION) {
                    v = fmin(1.0, S);
                    ps = S < 1.0;
                } else if (op == SG_OP_INTERSECTION) {
                    const double nm1 = P.node_nm1[k];
                    v = fmax(nm1, S) - nm1;
                    ps = S > nm1;
                } else {
                    v = fmax(0.0, S);
                    ps = S > 0.0;
                }
                if (ps) passm |= 1u << k;
                if (k == root) s = v;
                const int par = P.node_parent[k];
#pragma unroll
                for (int j = k + 1; j < NN; ++j)
                    if (par == j) acc[j] += P.node_sign[k] * v;
#pragma unroll
                for (int g = 0; g < NN; ++g)
                    if (g < P.nlev && P.lev_node[g] == k) lvv[g] = v;
            }
        }
        if (lev_root) {
            // Alg. cap: s = v_0, s = min{1, q_g s + v_g}; d s / d v_g =
            // pass_g prod_{j > g} pass_j q_j (d s / d v_0 = prod_{j >= 1} pass_j q_j)
            uint32_t lpass = 0u;
            double t = lvv[0];
#pragma unroll
            for (int g = 1; g < NN; ++g) {
                if (g < P.nlev) {
                    const double x = P.lev_q[g] * t + lvv[g];
                    if (x < 1.0) lpass |= 1u << g;
                    t = fmin(1.0, x);
                }
            }
            s = t;
            double a = 1.0;
#pragma unroll
            for (int g = NN - 1; g >= 1; --g) {
                if (g < P.nlev) {
                    const double pg = ((lpass >> g) & 1u) ? 1.0 : 0.0;
                    const double rg = a * pg;
                    a *= pg * P.lev_q[g];
#pragma unroll
                    for (int j = 0; j < NN; ++j)
                        if (P.lev_node[g] == j) r[j] = rg;
                }
            }
#pragma unroll
            for (int j = 0; j < NN; ++j)
                if (P.lev_node[0] == j) r[j] = a;
        } else {
#pragma unroll
            for (int k = 0; k < NN; ++k)
                if (k == root) r[k] = 1.0;
        }
        o.s = s;
        // reverse: parents come after their children, so walking down from
        // the root every r[parent] is final before it is used
#pragma unroll
        for (int k = NN - 2; k >= 0; --k) {
            if (k < root) {
                const int par = P.node_parent[k];
                if (!(lev_root && par == root)) {
                    double rp = 0.0;
#pragma unroll
                    for (int j = k + 1; j < NN; ++j)
                        if (par == j) rp = ((passm >> j) & 1u) ? r[j] : 0.0;
                    r[k] = rp * P.node_sign[k];
                }
            }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            o.cf[c] = 0.0;
            if (c < P.nclass) {
                const int kn = P.cls_node[c];
#pragma unroll
                for (int k = 0; k < NN; ++k)
                    if (kn == k) o.cf[c] = ((passm >> k) & 1u) ? r[k] * P.cls_sign[c] : 0.0;
            }
        }
        return o;
    }
}


// Coordinates of the kBlock samples of a tile in LDS, [4][kBlock]: centers and
// widths along u, then along v.
struct SampleLat {
    const double* p;
    __device__ double uc(int t) const { return p[t]; }
    __device__ double uw(int t) const { return p[kBlock + t]; }
    __device__ double vc(int t) const { return p[2 * kBlock + t]; }
    __device__ double vw(int t) const { return p[3 * kBlock + t]; }
};

// Partials of a convex polygon at one sample, times a; one reduction per
// vertex field and edge.
template <int SIGS>
__device__ __forceinline__ void poly_partials(const KParams& P, const DevPrim& pr, const FieldWin& fwx,
                                              const FieldWin& fwy, double ad, double uc, double vc) {
    const int N = uniform_int(pr.nvert);
    const ConstF64 xs = const_space<ConstF64>(P.fval + uniform_int(pr.f0));
    const ConstF64 ys = xs + N;
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
        emit_win(P, fwx, pr.f0 + i, (float)(g * ((ey - wy) * iL + dL2 * ex)));
        emit_win(P, fwy, pr.f0 + N + i, (float)(g * ((wx - ex) * iL + dL2 * ey)));
        emit_win(P, fwx, pr.f0 + j, (float)(g * (wy * iL - dL2 * ex)));
        emit_win(P, fwy, pr.f0 + N + j, (float)(g * (-wx * iL - dL2 * ey)));
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
__device__ __forceinline__ void gcart_partials(const KParams& P, const DevPrim& pr, const float* sAc, const SampleLat& L,
                               const Tile& T, int comp, int u0, float* sg) {
    constexpr int Q = kBlock / 64;
    const int lane = threadIdx.x & 63;
    const int TU = P.tu;
    const double* fv = P.fval;
    const int M = pr.nvert;
    const double* yp = fv + pr.f0 + 2;
    const double* ym = yp + M;
    const GSeg* gs = P.gseg + pr.gs0 + (int64_t)comp * P.nu;
    const int jlo = gs[u0].j, jhi = gs[min(u0 + TU, P.nu) - 1].j;   // segments of the tile's first / last sample
    const int nvx = jhi - jlo + 2;               // vertices jlo .. jhi + 1
    // (the LDS buckets add lanes' FP32 values in hardware order: not in deterministic mode)
    const bool bucket = nvx <= kSegBucket && !P.fx;
    if (bucket) {
        for (int i = lane; i < 2 * nvx; i += 64) sg[i] = 0.0f;
        __builtin_amdgcn_s_waitcnt(0xc07f);      // lgkmcnt(0): the zeros are in LDS
        __builtin_amdgcn_wave_barrier();
    }
    const double xs0 = fv[pr.f0], xs1 = fv[pr.f0 + 1];
    double sxs = 0.0, sxe = 0.0;
#pragma unroll 1
    for (int q = 0; q < Q; ++q) {
        const int t = q * 64 + lane;
        const float a = sAc[t];
        if (__ballot(a != 0.0f) == 0) continue;
        const double uc = L.uc(t), uw = L.uw(t), vc = L.vc(t), vw = L.vw(t);
        const double ad = (double)a;
        float c0 = 0.0f, c1 = 0.0f, c2 = 0.0f, c3 = 0.0f;
        int j = 0;
        if (a != 0.0f) {
            double rx, drx0, drx1;
            rect_vd<SIGS>(pr.sk0, kval(pr.sm0, pr.k0, uw), uc, xs0, xs1, rx, drx0, drx1);
            const GSeg sgm = gs[min(u0 + (t & (TU - 1)), P.nu - 1)];
            j = sgm.j;
            const double t01 = sgm.t;
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

// Partials of a Fourier-radius boundary, times the column sums, over the
// kBlock samples of the tile handled by this wavefront.  d (R - r) / d x0 =
// R'(theta) sin(theta) / r + cos(theta) (and the y0 pair), d / d R0 = 1,
// d / d c_n = -cos n theta, d / d s_n = -sin n theta.  The coefficient sums go
// through polar_emit, which combines candidates that share a coefficient's
// parameter (a global shape coefficient) in the block's LDS.
constexpr int kPolarSlots = 64;     // >= 2 x the largest Fourier order

// Adds the wavefront sum of v for coefficient field `field` (slot = its
// position among the coefficients): into the block's LDS slot when the slot
// holds, or can be claimed for, the field's parameter; else to grad directly.
__device__ __forceinline__ void polar_emit(const KParams& P, const FieldWin& w, int field, int slot, float v,
                                           double* s_pacc, int* s_pkey) {
    int idx;
    double b;
    win_ref(w, field, idx, b);
    if (idx < 0) return;
    if (__ballot(v != 0.0f) == 0) return;
    const float sum = wave_sum(v);
    if ((threadIdx.x & 63) == 0) {
        if (P.fx) {       // deterministic mode: no LDS combining (FP64 LDS atomics add in any order)
            grad_add(P, idx, b * (double)sum);
            return;
        }
        int k = s_pkey[slot];
        if (k == -2) {
            const int old = atomicCAS(&s_pkey[slot], -2, idx);
            k = (old == -2) ? idx : old;
        }
        if (k == idx) atomicAdd(&s_pacc[slot], b * (double)sum);
        else atomicAdd(grad_copy(P) + idx, b * (double)sum);
    }
}

// A wavefront's per-lane sums of the Fourier-coefficient partials over the
// candidates it has processed, while they are of one coefficient group (the
// same coefficient fields: the global shape coefficients of a lattice of
// scatterers): one reduction per coefficient per wavefront instead of one
// per candidate.  The group's coefficient values (coef, one per lane) and
// field window (kw, its coefficient lanes) are read once per group; n = 0:
// empty.  Orders above kAccN take the per-candidate reductions.
constexpr int kAccN = 6;
struct PolarAcc {
    float c[kAccN], s[kAccN];
    int n, grp;
    float coef;
    FieldWin kw;
};
__device__ __forceinline__ void polar_acc_clear(PolarAcc& a) { a.n = 0; }

// Reduces and emits the accumulated sums (then empty): the 2 kAccN sums of
// every lane in one reduce-scatter, after which lane l < 2 kAccN holds sum l
// (c_1..c_kAccN, then s_1..s_kAccN) and emits it as polar_emit would: into
// the block's LDS slot of its coefficient when the slot holds, or can be
// claimed for, its parameter, else to grad.
__device__ __forceinline__ void polar_acc_flush(const KParams& P, PolarAcc& a, double* s_pacc, int* s_pkey) {
    const int N = a.n;
    if (N == 0) return;
    const int lane = threadIdx.x & 63;
    float v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = k < kAccN ? a.c[k] : (k < 2 * kAccN ? a.s[k - kAccN] : 0.0f);
    row_scatter_sum<8, 0x140>(v, lane);
    row_scatter_sum<4, 0x141>(v, lane);
    row_scatter_sum<2, 0x1B>(v, lane);
    row_scatter_sum<1, 0xB1>(v, lane);
    float tot = v[0] + __shfl_xor(v[0], 16, 64);
    tot += __shfl_xor(tot, 32, 64);
    const int l = lane & 15;
    const int n = l < kAccN ? l : l - kAccN;                // order - 1
    const int slot = l < kAccN ? n : N + n;                  // position among the 2 N coefficients
    const bool valid = lane < 2 * kAccN && n < N;
    const int src = 3 + (valid ? slot : 0);                  // the coefficient's lane in the window
    const int idx = __shfl(a.kw.idx, src, 64);
    const double b = __shfl(a.kw.b, src, 64);
    if (valid && idx >= 0 && tot != 0.0f) {
        const double val = b * (double)tot;
        if (P.fx) {       // deterministic mode: no LDS combining (FP64 LDS atomics add in any order)
            grad_add(P, idx, val);
        } else {
            int k = s_pkey[slot];
            if (k == -2) {
                const int old = atomicCAS(&s_pkey[slot], -2, idx);
                k = (old == -2) ? idx : old;
            }
            if (k == idx) atomicAdd(&s_pacc[slot], val);
            else atomicAdd(grad_copy(P) + idx, val);
        }
    }
    a.n = 0;
}

// polar_partials into the running sums (order N <= kAccN): x0 y0 R0 and
// their references come from the staged record, the coefficients from the
// group's registers; one sample at a time, the radius recurrence keeps each
// cos / sin (n theta) for the coefficient partials once d F / d (R - r) is
// known, so the rotation runs once per sample.
template <int SIGS>
__device__ __forceinline__ void polar_partials_acc(const KParams& P, const PrimRec& cr, const float* sAc,
                                                   const SampleLat& L, double* s_pacc, int* s_pkey, PolarAcc& acc) {
    constexpr int Q = kBlock / 64;
    const int lane = threadIdx.x & 63;
    const DevPrim& pr = cr.pr;
    const int N = uniform_int(pr.nvert);
    const int grp = uniform_int(pr.cgrp);
    if (acc.n == 0 || acc.grp != grp) {
        polar_acc_flush(P, acc, s_pacc, s_pkey);
        load_win(P, acc.kw, pr.f0, pr.f0 + 3 + 2 * N);
        acc.coef = lane < 2 * N ? (float)P.fval[pr.f0 + 3 + lane] : 0.0f;
        acc.n = N;
        acc.grp = grp;
#pragma unroll
        for (int n = 0; n < kAccN; ++n) acc.c[n] = acc.s[n] = 0.0f;
    }
    const float k0 = (float)pr.k0;
    float an[kAccN], bn[kAccN];
#pragma unroll
    for (int n = 0; n < kAccN; ++n) {
        const int l = max(min(n, N - 1), 0);
        an[n] = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, acc.coef), l));
        bn[n] = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, acc.coef), N + l));
    }
    const double x0 = cr.f[0], y0 = cr.f[1];
    const float R0 = (float)cr.f[2];
    float sx = 0.0f, sy = 0.0f, sR = 0.0f;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int t = q * 64 + lane;
        const float av = sAc[t];
        if (__ballot(av != 0.0f) == 0) continue;
        float c1 = 1.0f, s1 = 0.0f, rv = 0.0f, iv = 0.0f;
        {
            const float dx = (float)(L.uc(t) - x0), dy = (float)(L.vc(t) - y0);
            rv = sqrtf(dx * dx + dy * dy);
            iv = rv > 0.0f ? 1.0f / rv : 0.0f;
            if (rv > 0.0f) {
                c1 = dx * iv;
                s1 = dy * iv;
            }
        }
        float cs[kAccN], sn[kAccN];
        float R = R0, dR = 0.0f, cn = 1.0f, snn = 0.0f;
#pragma unroll
        for (int n = 1; n <= kAccN; ++n) {
            const float crt = cn * c1 - snn * s1;
            snn = snn * c1 + cn * s1;
            cn = crt;
            cs[n - 1] = cn;
            sn[n - 1] = snn;
            if (n <= N) {
                R -= an[n - 1] * cn + bn[n - 1] * snn;
                dR += (float)n * (an[n - 1] * snn - bn[n - 1] * cn);
            }
        }
        float gg = 0.0f;
        if (av != 0.0f) {
            gg = av * k0 * sig_d32(pr.sk0, k0 * (R - rv));     // a * d F / d (R - r)
            if (rv > 0.0f) {
                sx += gg * (dR * s1 * iv + c1);
                sy += gg * (-dR * c1 * iv + s1);
            }
            sR += gg;
        }
#pragma unroll
        for (int n = 0; n < kAccN; ++n) {
            if (n < N) {
                acc.c[n] -= gg * cs[n];
                acc.s[n] -= gg * sn[n];
            }
        }
    }
    emit_ref(P, cr.fidx[0], cr.fb[0], sx);
    emit_ref(P, cr.fidx[1], cr.fb[1], sy);
    emit_ref(P, cr.fidx[2], cr.fb[2], sR);
}

template <int SIGS>
__device__ __forceinline__ void polar_partials(const KParams& P, const DevPrim& pr, const float* sAc,
                                               const SampleLat& L, double* s_pacc, int* s_pkey) {
    constexpr int Q = kBlock / 64;
    const int lane = threadIdx.x & 63;
    const int N = uniform_int(pr.nvert);
    FieldWin w;           // x0, y0, R0, c_1..c_N, s_1..s_N: 2 N + 3 <= 61 fields
    load_win(P, w, pr.f0, pr.f0 + 3 + 2 * N);
    const double* f = P.fval + pr.f0;
    const float k0 = (float)pr.k0;
    // the 2 N coefficients, one per lane (c_1..c_N, then s_1..s_N), read by
    // lane moves in the per-sample recurrence instead of a load per term
    const float coef = lane < 2 * N ? (float)f[3 + lane] : 0.0f;
    const float R0 = (float)f[2];
    float g[Q], c1[Q], s1[Q];
    float sx = 0.0f, sy = 0.0f, sR = 0.0f;
    // derivatives only: FP32 after the FP64 differences (as for the ellipse;
    // k (R - r) keeps ~1e-6 absolute).  The Fourier recurrence runs over the
    // terms outside and the wavefront's Q samples inside, so each coefficient
    // is read once per candidate.
    float av[Q], rv[Q], iv[Q], R[Q], dR[Q], cn[Q], sn[Q];
    bool rowlive[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int t = q * 64 + lane;
        av[q] = sAc[t];
        rowlive[q] = __ballot(av[q] != 0.0f) != 0;
        c1[q] = 1.0f;
        s1[q] = 0.0f;
        rv[q] = 0.0f;
        iv[q] = 0.0f;
        if (rowlive[q]) {
            const float dx = (float)(L.uc(t) - f[0]), dy = (float)(L.vc(t) - f[1]);
            rv[q] = sqrtf(dx * dx + dy * dy);
            iv[q] = rv[q] > 0.0f ? 1.0f / rv[q] : 0.0f;
            if (rv[q] > 0.0f) {
                c1[q] = dx * iv[q];
                s1[q] = dy * iv[q];
            }
        }
        R[q] = R0;
        dR[q] = 0.0f;
        cn[q] = 1.0f;
        sn[q] = 0.0f;
    }
    for (int n = 1; n <= N; ++n) {
        const float an = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, coef), n - 1));
        const float bn = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, coef), N + n - 1));
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const float cr = cn[q] * c1[q] - sn[q] * s1[q];
            sn[q] = sn[q] * c1[q] + cn[q] * s1[q];
            cn[q] = cr;
            R[q] -= an * cn[q] + bn * sn[q];
            dR[q] += (float)n * (an * sn[q] - bn * cn[q]);
        }
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        g[q] = 0.0f;
        if (av[q] != 0.0f) {
            const float gg = av[q] * k0 * sig_d32(pr.sk0, k0 * (R[q] - rv[q]));     // a * d F / d (R - r)
            if (rv[q] > 0.0f) {
                sx += gg * (dR[q] * s1[q] * iv[q] + c1[q]);
                sy += gg * (-dR[q] * c1[q] * iv[q] + s1[q]);
            }
            sR += gg;
            g[q] = gg;
        }
    }
    emit_win(P, w, pr.f0, sx);
    emit_win(P, w, pr.f0 + 1, sy);
    emit_win(P, w, pr.f0 + 2, sR);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        cn[q] = 1.0f;
        sn[q] = 0.0f;
    }
    for (int n = 1; n <= N; ++n) {
        float pc = 0.0f, ps = 0.0f;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const float c = cn[q] * c1[q] - sn[q] * s1[q];
            sn[q] = sn[q] * c1[q] + cn[q] * s1[q];
            cn[q] = c;
            pc -= g[q] * cn[q];
            ps -= g[q] * sn[q];
        }
        polar_emit(P, w, pr.f0 + 2 + n, n - 1, pc, s_pacc, s_pkey);
        polar_emit(P, w, pr.f0 + 2 + N + n, N + n - 1, ps, s_pacc, s_pkey);
    }
}

// Partials of a Polar2D boundary, times the column sums, over the kBlock
// samples of the tile handled by this wavefront: with t = k (R(theta) - r),
// R(theta) = R (1 + delta cos(alpha theta)), d / d R = 1 + delta cos(alpha
// theta), d / d delta = R cos(alpha theta), and the center pair as for the
// Fourier radius with R'(theta) = -R delta alpha sin(alpha theta).  FP32 after
// the FP64 coordinate differences.
template <int SIGS>
__device__ __forceinline__ void polar2d_partials(const KParams& P, const DevPrim& pr, const float* sAc,
                                                 const SampleLat& L) {
    constexpr int Q = kBlock / 64;
    const int lane = threadIdx.x & 63;
    const int A = uniform_int(pr.nvert);
    FieldWin w;           // x0, y0, R, delta
    load_win(P, w, pr.f0, pr.f0 + 4);
    const double* f = P.fval + pr.f0;
    const float k0 = (float)pr.k0;
    const float R = (float)f[2], dl = (float)f[3];
    float sx = 0.0f, sy = 0.0f, sR = 0.0f, sd = 0.0f;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int t = q * 64 + lane;
        const float a = sAc[t];
        if (__ballot(a != 0.0f) == 0) continue;
        if (a != 0.0f) {
            const float dx = (float)(L.uc(t) - f[0]), dy = (float)(L.vc(t) - f[1]);
            const float r = sqrtf(dx * dx + dy * dy);
            const float ir = r > 0.0f ? 1.0f / r : 0.0f;
            const float c1 = r > 0.0f ? dx * ir : 1.0f, s1 = r > 0.0f ? dy * ir : 0.0f;
            float cn = 1.0f, sn = 0.0f;
            for (int n = 0; n < A; ++n) {
                const float c = cn * c1 - sn * s1;
                sn = sn * c1 + cn * s1;
                cn = c;
            }
            const float Rth = R * (1.0f + dl * cn);
            const float dR = -R * dl * (float)A * sn;
            const float gg = a * k0 * sig_d32(pr.sk0, k0 * (Rth - r));     // a * d F / d (R(theta) - r)
            if (r > 0.0f) {
                sx += gg * (dR * s1 * ir + c1);
                sy += gg * (-dR * c1 * ir + s1);
            }
            sR += gg * (1.0f + dl * cn);
            sd += gg * R * cn;
        }
    }
    emit_win(P, w, pr.f0, sx);
    emit_win(P, w, pr.f0 + 1, sy);
    emit_win(P, w, pr.f0 + 2, sR);
    emit_win(P, w, pr.f0 + 3, sd);
}

// Partials of the taper's sine-series boundary, times the column sums, over
// the kBlock samples of the tile handled by this wavefront: the x-range pair
// like a Rect1D, and d F / d v_i = (d F / d f) envelope(x) sin(i phi), the
// sines by repeated FP32 rotation (error linear in i), the terms reduced 16 at
// a time; a wavefront whose samples all have d F / d f = 0 skips the terms.
template <int SIGS, int Q>
__device__ __forceinline__ void series_partials(const KParams& P, const DevPrim& pr, const float* sAc,
                                                const SampleLat& L, int qbase) {
    const int lane = threadIdx.x & 63;
    const double* fv = P.fval;
    const double* c = P.consts + pr.c0;
    FieldWin fw;          // xs, xe
    load_win(P, fw, pr.f0, pr.f0 + 2);
    float w[Q], s1[Q], c1[Q];
    float sxs = 0.0f, sxe = 0.0f;
    bool any = false;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int t = (qbase + q) * 64 + lane;
        const float a = sAc[t];
        w[q] = 0.0f;
        s1[q] = 0.0f;
        c1[q] = 1.0f;
        if (a != 0.0f) {
            const double uc = L.uc(t), vc = L.vc(t);
            double rx, drx0, drx1;
            rect_vd<SIGS>(pr.sk0, kval(pr.sm0, pr.k0, L.uw(t)), uc, fv[pr.f0], fv[pr.f0 + 1], rx, drx0, drx1);
            double env, sn, cs;
            const double f = series_f(pr, fv, c, uc, &env, &sn, &cs);
            const double ky = kval(pr.sm1, pr.k1, L.vw(t)), yr = vc - c[4];
            double sp, dsp, sm, dsm;
            sig_vd<SIGS>(pr.sk1, ky * (f - yr), sp, dsp);
            sig_vd<SIGS>(pr.sk1, ky * (f + yr), sm, dsm);
            const double ad = (double)a;
            sxs += (float)(ad * drx0 * sp * sm);
            sxe += (float)(ad * drx1 * sp * sm);
            const double gf = ad * rx * ky * (dsp * sm + sp * dsm);    // a * d F / d f
            w[q] = (float)(gf * env);
            s1[q] = (float)sn;
            c1[q] = (float)cs;
            any = any || (w[q] != 0.0f);
        }
    }
    emit_win(P, fw, pr.f0, sxs);
    emit_win(P, fw, pr.f0 + 1, sxe);
    if (__ballot(any) == 0) return;
    float si[Q], ci[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        si[q] = s1[q];
        ci[q] = c1[q];
    }
    // the terms 16 at a time: each lane forms its products for 16 terms, a
    // reduce-scatter over each 16-lane row (four DPP exchanges, one term
    // index bit each) leaves term (lane mod 16)'s row sum in the lane, two
    // cross-row exchanges complete the wavefront sums, and lanes 0-15 add
    // their terms together (about 3 instructions per term where a wavefront
    // reduction and an atomic each took about 15)
    for (int i0 = 0; i0 < pr.nvert; i0 += 16) {
        const int term = i0 + (lane & 15);
        sg_field r{0.0, 0.0, -1};
        if (lane < 16 && term < pr.nvert) r = P.fref[pr.f0 + 2 + term];
        float a[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            float acc = 0.0f;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                acc += w[q] * si[q];
                const float sn = si[q] * c1[q] + ci[q] * s1[q];
                ci[q] = ci[q] * c1[q] - si[q] * s1[q];
                si[q] = sn;
            }
            a[k] = acc;
        }
        row_scatter_sum<8, 0x140>(a, lane);    // row_mirror: lane i <-> 15 - i
        row_scatter_sum<4, 0x141>(a, lane);    // row_half_mirror: i <-> 7 - i within 8
        row_scatter_sum<2, 0x1B>(a, lane);     // quad_perm [3,2,1,0]
        row_scatter_sum<1, 0xB1>(a, lane);     // quad_perm [1,0,3,2]
        float tot = a[0] + __shfl_xor(a[0], 16, 64);
        tot += __shfl_xor(tot, 32, 64);
        if (r.idx >= 0 && tot != 0.0f) grad_add(P, (int)r.idx, r.b * (double)tot);
    }
}

// One candidate primitive, handled by one wavefront for all kBlock samples of
// the block's tile (kBlock / 64 samples per lane): in-plane partials times the
// class column sums sAc[sample], summed over the lane's samples, reduced over
// the wavefront, and added with one atomic per parameter field.
template <int TYPES, int SIGS>
__device__ __forceinline__ void block_partials(const KParams& P, const PrimRec& cr, const float* sAc, const SampleLat& L,
                               const Tile& T, int comp, int u0, float* sg, double* s_pacc, int* s_pkey,
                               PolarAcc& acc) {
    constexpr int Q = kBlock / 64;
    const int lane = threadIdx.x & 63;
    const DevPrim& pr = cr.pr;
    const int type = (TYPES == T_BOX) ? SG_PRIM_BOX : pr.type;
    if constexpr ((TYPES & T_BOX) != 0) {
        if (type == SG_PRIM_BOX) {
            const double u0 = cr.f[0], u1 = cr.f[1], v0 = cr.f[2], v1 = cr.f[3];
            double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int t = q * 64 + lane;
                const float a = sAc[t];
                if (a != 0.0f) {
                    const double ad = (double)a;
                    double ru = 1.0, du0 = 0.0, du1 = 0.0, rv = 1.0, dv0 = 0.0, dv1 = 0.0;
                    if (pr.ubnd) rect_vd<SIGS>(pr.sk0, kval(pr.sm0, pr.k0, L.uw(t)), L.uc(t), u0, u1, ru, du0, du1);
                    if (pr.vbnd) rect_vd<SIGS>(pr.sk1, kval(pr.sm1, pr.k1, L.vw(t)), L.vc(t), v0, v1, rv, dv0, dv1);
                    s0 += ad * du0 * rv;
                    s1 += ad * du1 * rv;
                    s2 += ad * ru * dv0;
                    s3 += ad * ru * dv1;
                }
            }
            if (pr.ubnd) {
                emit_ref(P, cr.fidx[0], cr.fb[0], (float)s0);
                emit_ref(P, cr.fidx[1], cr.fb[1], (float)s1);
            }
            if (pr.vbnd) {
                emit_ref(P, cr.fidx[2], cr.fb[2], (float)s2);
                emit_ref(P, cr.fidx[3], cr.fb[3], (float)s3);
            }
            return;
        }
    }
    if constexpr ((TYPES & T_ELL) != 0) {
        if (type == SG_PRIM_ELLIPSE) {
            const double x0 = cr.f[0], y0 = cr.f[1], r = cr.f[2];
            const double rhi = r + pr.reach0, rlo = r - pr.reach0;
            double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int t = q * 64 + lane;
                const float a = sAc[t];
                if (a != 0.0f) {
                    const double qx = (L.uc(t) - x0) * pr.iax, qy = (L.vc(t) - y0) * pr.iay;
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
            emit_ref(P, cr.fidx[0], cr.fb[0], (float)s0);
            emit_ref(P, cr.fidx[1], cr.fb[1], (float)s1);
            emit_ref(P, cr.fidx[2], cr.fb[2], (float)s2);
            return;
        }
    }
    if constexpr ((TYPES & T_POLY) != 0) {
        if (type == SG_PRIM_POLY) {
            FieldWin fwx, fwy;    // the x and y vertex fields (nvert <= 64)
            load_win(P, fwx, pr.f0, pr.f0 + pr.nvert);
            load_win(P, fwy, pr.f0 + pr.nvert, pr.f0 + 2 * pr.nvert);
#pragma unroll 1
            for (int q = 0; q < Q; ++q) {
                const int t = q * 64 + lane;
                const float a = sAc[t];
                if (__ballot(a != 0.0f) == 0) continue;
                poly_partials<SIGS>(P, pr, fwx, fwy, (double)a, L.uc(t), L.vc(t));
            }
            return;
        }
    }
    if constexpr ((TYPES & T_GCART) != 0) {
        if (type == SG_PRIM_GCART) {
            gcart_partials<SIGS>(P, pr, sAc, L, T, comp, u0, sg);
            return;
        }
    }
    if constexpr ((TYPES & T_POLAR) != 0) {
        if (type == SG_PRIM_POLAR2D) {
            polar2d_partials<SIGS>(P, pr, sAc, L);
            return;
        }
        if (type == SG_PRIM_POLAR) {
            // the running sums only in the Fourier feature set (the catch-all
            // kernel has no registers to spare for them)
            if constexpr (TYPES == (T_BOX | T_POLAR)) {
                if (pr.nvert <= kAccN) {
                    polar_partials_acc<SIGS>(P, cr, sAc, L, s_pacc, s_pkey, acc);
                    return;
                }
            }
            polar_partials<SIGS>(P, pr, sAc, L, s_pacc, s_pkey);
            return;
        }
    }
    // sine-series boundaries: series_split, called by every wavefront
}

// The sine-series candidates of a staged set: every wavefront takes its own
// 64 samples of each (one candidate's K term reductions would otherwise run on
// one wavefront while the other three wait at the block's end).
template <int TYPES, int SIGS>
__device__ __forceinline__ void series_split(const KParams& P, const PrimRec* s_rec, int n, const float* sA,
                                             const SampleLat& L) {
    if constexpr ((TYPES & T_SERIES) != 0) {
        const int wave = threadIdx.x >> 6;
        for (int j = 0; j < n; ++j)
            if (s_rec[j].pr.type == SG_PRIM_SERIES)
                series_partials<SIGS, 1>(P, s_rec[j].pr, sA + s_rec[j].pr.cls * kBlock, L, wave);
    }
}

// ------------------------------------------------------------------ tiles
// In-plane tile of a block: kBlock samples, tu x tv, and its wavefronts' sub-tiles.
struct TileGeom {
    int comp, u, v, uu, vv;
    bool act;
    double uc, uw, vc, vw;
    Tile T;
};

// Linear tiles: the block's samples are in-plane indices [i0, i0 + 256) in
// row-major order; a span of indices covers the u range of its rows (the
// whole row width when it crosses a row end).
__device__ __forceinline__ void span_box(const KParams& P, const double* ucs, const double* vcs, int first, int last,
                                         double& ulo, double& uhi, double& vlo, double& vhi) {
    const int v0 = first / P.nu, v1 = last / P.nu;
    const int u0 = (v0 == v1) ? first - v0 * P.nu : 0;
    const int u1 = (v0 == v1) ? last - v1 * P.nu : P.nu - 1;
    ulo = ucs[u0];
    uhi = ucs[u1];
    vlo = vcs[v0];
    vhi = vcs[v1];
}

template <bool LINEAR = false>
__device__ __forceinline__ TileGeom tile_geom(const KParams& P, int b) {
    const int tid = threadIdx.x, wave = tid >> 6;
    TileGeom G;
    if (LINEAR && P.linear) {
        const int nuv = P.nu * P.nv;
        const int ti = b % P.tiles_u;
        G.comp = b / P.tiles_u;
        const int first = ti * kBlock, last = min(first + kBlock, nuv) - 1;
        const int idx = first + tid;
        G.act = idx < nuv;
        const int ic = min(idx, nuv - 1);
        G.vv = ic / P.nu;
        G.uu = ic - G.vv * P.nu;
        G.u = G.act ? G.uu : P.nu;
        G.v = G.vv;
        const double* __restrict__ ucs = P.uc[G.comp];
        const double* __restrict__ vcs = P.vc[G.comp];
        G.uc = ucs[G.uu];
        G.uw = P.uw[G.comp][G.uu];
        G.vc = vcs[G.vv];
        G.vw = P.vw[G.comp][G.vv];
        Tile& T = G.T;
        span_box(P, ucs, vcs, first, last, T.ulo, T.uhi, T.vlo, T.vhi);
        const int wf = first + wave * 64;
        T.wave_live = wf < nuv;
        span_box(P, ucs, vcs, min(wf, nuv - 1), min(wf + 64, nuv) - 1, T.wulo, T.wuhi, T.wvlo, T.wvhi);
        return G;
    }
    // row-major tile order: consecutive blocks are side by side in u, so a
    // range of blocks covers whole rows (taper VJP 131.1 -> 130.5 us against
    // v first)
    const int tui = b % P.tiles_u;
    b /= P.tiles_u;
    const int tvi = b % P.tiles_v;
    G.comp = b / P.tiles_v;
    const int TU = P.tu;
    G.u = tui * TU + (tid & (TU - 1));
    G.v = tvi * P.tv + tid / TU;
    G.act = (G.u < P.nu) && (G.v < P.nv);
    G.uu = min(G.u, P.nu - 1);
    G.vv = min(G.v, P.nv - 1);
    const double* __restrict__ ucs = P.uc[G.comp];
    const double* __restrict__ vcs = P.vc[G.comp];
    G.uc = ucs[G.uu];
    G.uw = P.uw[G.comp][G.uu];
    G.vc = vcs[G.vv];
    G.vw = P.vw[G.comp][G.vv];
    const int u0 = tui * TU, u1 = min(u0 + TU, P.nu) - 1;
    const int v0 = tvi * P.tv, v1 = min(v0 + P.tv, P.nv) - 1;
    Tile& T = G.T;
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
    return G;
}

// ------------------------------------------------------------------ column kernel
// Tables every wavefront reads at the same address (step and group codes,
// extrusion tables) are read through the constant address space (ConstU32,
// ConstF64): scalar loads, which neither occupy vector registers nor wait
// behind the field loads.

// Raw buffer resource over [base, base + bytes) (bytes clamped to 32 bits;
// reads past the end return 0).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void* base, int64_t bytes) {
    const int32_t n = bytes <= 0 ? 0 : (bytes >= 0xFFFFFFFFll ? (int32_t)0xFFFFFFFF : (int32_t)(uint32_t)bytes);
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, n, 0x00020000);
}

// First and last group of a component whose code is nonzero (some class at
// nonzero extrusion, or a general step); ghi < glo when there is none.  Every
// wavefront computes it (the codes are few and cached), up to 256 codes per
// memory round trip.
__device__ __forceinline__ void live_groups(const uint32_t* __restrict__ gc, int ngw, int& glo, int& ghi) {
    const int lane = threadIdx.x & 63;
    glo = ngw;
    ghi = -1;
    for (int base = 0; base < ngw; base += 256) {
        uint32_t c[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int i = base + k * 64 + lane;
            c[k] = (i < ngw) ? gc[i] : 0u;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint64_t m = __ballot(c[k] != 0u);
            if (m != 0) {
                glo = min(glo, base + k * 64 + __ffsll((unsigned long long)m) - 1);
                ghi = max(ghi, base + k * 64 + 63 - __clzll((long long)m));
            }
        }
    }
    glo = uniform_int(glo);
    ghi = uniform_int(ghi);
}

// One block = one in-plane tile of kBlock samples (tu x tv) of one component
// and one segment [w0, w1) of the column (w0 a multiple of kGroup); one thread
// per sample.
//  1. The first set of field loads goes out; the candidate primitives of the
//     tile are listed and their records staged in LDS; each thread sums the
//     in-plane factors per extrusion class, F_c (FP64).
//  2. The column is streamed.  On a "binary" step every class factor Z_c(w)
//     is exactly 0 or 1 (and the w-bound derivatives of classes with
//     column-axis parameters vanish): its composition depends only on F and
//     on the mask of classes at 1.  Along a run of equal masks the column sums
//     A_c = sum_w g(w) d eps/d s_c Z_c(w) therefore factor into (d eps/d s_c
//     at that mask) x (sum of g over the run), and eps is one value per run.
//     Other steps are composed one by one.  Groups of kGroup binary steps with
//     one mask take a path with no per-step decisions.
//  3. (VJP) A_c goes to LDS and the candidates are split over the wavefronts:
//     in-plane partials times A_c over the tile's samples, reduced over the
//     wavefront, one FP64 atomic per (wavefront, parameter field).
template <int MODE, int TREE, int TYPES, int SIGS>
__device__ __forceinline__ void column_body(const KParams& P, int b) {
    constexpr int NC = tree_nc(TREE);
    constexpr bool SPARSE = (MODE == MODE_VJP_SPARSE);
    constexpr bool FDM = (MODE == MODE_FD || MODE == MODE_FD_SPARSE);     // two evaluation points
    constexpr bool FIELDS = (MODE == MODE_VJP_FIELDS) || SPARSE;
    constexpr bool VJP = FIELDS || (MODE == MODE_VJP_GEPS);
    constexpr int U = (MODE == MODE_VJP_GEPS) ? 8 : 4;      // steps per load set (multiple of kGroup)
    constexpr int NG = U / kGroup;
    constexpr int EB = FIELDS ? 8 : 4;                       // bytes per sample of the streamed planes
    __shared__ int s_cand[kCandCap];
    __shared__ int s_cnt[kScanCnt];
    __shared__ PrimRec s_rec[kStageRec];
    __shared__ float sA[VJP ? NC * kBlock : 1];
    __shared__ double s_lat[VJP ? 4 * kBlock : 1];
    __shared__ float sG[(VJP && (TYPES & T_GCART)) ? (kBlock / 64) * 2 * kSegBucket : 1];
    __shared__ double s_pacc[(VJP && (TYPES & T_POLAR)) ? kPolarSlots : 1];
    __shared__ int s_pkey[(VJP && (TYPES & T_POLAR)) ? kPolarSlots : 1];
    const int tid = threadIdx.x, wave = tid >> 6;

    // block b: tile b mod ntile of segment b / ntile, so the blocks in flight
    // read one compact window (every tile at the same column steps; the 2D
    // grating's 16 segments per tile: VJP 30.5 -> 28.5 us against segment-
    // fastest order)
    const int ntile = P.ncomp * P.tiles_u * P.tiles_v;
    const int seg = b / ntile, tile = b - seg * ntile;
    const TileGeom G = tile_geom<MODE == MODE_EPS>(P, tile);     // linear tiles: eps_build only
    const int comp = G.comp;
    const bool act = G.act;
    const int ngw = (P.nw + kGroup - 1) / kGroup;
    int w0 = seg * P.seglen;
    int w1 = min(w0 + P.seglen, P.nw);
    if constexpr (SPARSE || MODE == MODE_FD_SPARSE) {
        if constexpr (MODE == MODE_FD_SPARSE) {
            // a tile that no primitive referencing the parameter reaches, at
            // either evaluation point, has no difference
            if (!P.fd_all) {
                const Tile& T = G.T;
                bool hit = false;
                const int j1 = P.kprim_off[P.fd_k + 1];
                for (int j = P.kprim_off[P.fd_k]; j < j1 && !hit; ++j) {
                    const int pi = P.kprim[j];
                    const float4 a = P.bbox[pi], c = P.bbox2[pi];
                    hit = ((double)a.x <= T.uhi && (double)a.y >= T.ulo && (double)a.z <= T.vhi && (double)a.w >= T.vlo) ||
                          ((double)c.x <= T.uhi && (double)c.y >= T.ulo && (double)c.z <= T.vhi && (double)c.w >= T.vlo);
                }
                if (!hit) return;
            }
        }
        // the segments split the component's steps from its first to its last
        // group with some class at nonzero extrusion (at either evaluation
        // point); a block whose segment is empty has nothing to add
        int glo, ghi;
        live_groups(P.gcode + (int64_t)comp * ngw, ngw, glo, ghi);
        if constexpr (MODE == MODE_FD_SPARSE) {
            int glo2, ghi2;
            live_groups(P.gcode2 + (int64_t)comp * ngw, ngw, glo2, ghi2);
            glo = min(glo, glo2);
            ghi = max(ghi, ghi2);
        }
        if (ghi < glo) return;
        const int lw0 = glo * kGroup, lw1 = min(P.nw, (ghi + 1) * kGroup);
        const int slen = ((lw1 - lw0 + P.nseg - 1) / P.nseg + kGroup - 1) / kGroup * kGroup;
        w0 = lw0 + seg * slen;
        w1 = min(w0 + slen, lw1);
        if (w0 >= w1) return;
    }
    const int64_t b0 = (int64_t)G.uu + (int64_t)G.vv * P.sv;     // offset within a column plane
    const uint32_t lane_off = (uint32_t)b0 * EB;
    const int64_t plane_bytes = P.plane * EB;
    const int64_t step_bytes = P.sw * EB;
    const ConstU32 gcode = const_space<ConstU32>(P.gcode + (int64_t)comp * ngw);
    const ConstU32 gcode2 = const_space<ConstU32>(P.gcode2 + (int64_t)comp * ngw);
    const ConstU32 code = const_space<ConstU32>(P.code + (int64_t)comp * P.nw);
    const ConstU32 code2 = const_space<ConstU32>(P.code2 + (int64_t)comp * P.nw);
    const int64_t zcomp = (int64_t)comp * P.nclass * P.nw * 3;
    const ConstF64 ztab = const_space<ConstF64>(P.ztab + zcomp);
    const ConstF64 ztab2 = const_space<ConstF64>(P.ztab2 + zcomp);

    // combined code of a group / step (both evaluations for the FD modes)
    auto combine = [&](uint32_t c0, uint32_t c1) -> uint32_t {
        if constexpr (FDM)
            return ((c0 | c1) & kCodeGeneral) ? kCodeGeneral : ((c0 & 0xFFu) | ((c1 & 0xFFu) << 8));
        else
            return c0;
    };
    auto group_code = [&](int w) -> uint32_t {
        const int gi = min(w / kGroup, ngw - 1);
        return combine(gcode[gi], FDM ? gcode2[gi] : 0u);
    };
    auto step_code = [&](int w) -> uint32_t { return combine(code[w], FDM ? code2[w] : 0u); };
    auto load_zt = [&](ConstF64 zt, int w, double (&Z)[NC]) {
#pragma unroll
        for (int c = 0; c < NC; ++c) Z[c] = (c < P.nclass) ? zt[3 * ((int64_t)c * P.nw + w)] : 0.0;
    };

    // Field loads: two register sets of U steps each, double-buffered.  The
    // buffer resource of a set starts at its first step, so every load of the
    // set is (lane offset, immediate step offset), and ends at the segment's
    // end: the loads the double buffer issues past it return 0 without
    // touching memory.
    const char* plane0 = nullptr;
    const char* plane1 = nullptr;
    if constexpr (FIELDS) {
        plane0 = reinterpret_cast<const char*>(P.ef[comp]);
        plane1 = reinterpret_cast<const char*>(P.ea[comp]);
    } else if constexpr (MODE == MODE_VJP_GEPS) {
        plane0 = reinterpret_cast<const char*>(P.geps + (int64_t)comp * P.plane);
    }
    typedef float v2f __attribute__((ext_vector_type(2)));
    struct Set {
        v2f e[U], a[U];
        float g[U];
        uint32_t gc[NG];
    };
    Set sa, sb;
    // Sparse: the lane offset the loads use (dead lanes of a live wavefront
    // read the first live lane's address, which adds no cache lines), the
    // group codes of the next set (prefetched one set ahead, so the zero-length
    // resource of a set whose groups all have every class at zero extrusion is
    // known without a wait), and the steps read.
    uint32_t lane_ld = lane_off;
    uint32_t nextc[NG];
    int nsteps = 0;
    auto load_set = [&](Set& st, int w) {
        const int64_t off = (int64_t)w * step_bytes;
        int64_t len = min(plane_bytes - off, (int64_t)(w1 - w) * step_bytes);
        if constexpr (SPARSE) {
            bool dead = true;
#pragma unroll
            for (int h = 0; h < NG; ++h) {
                st.gc[h] = nextc[h];
                dead = dead && (nextc[h] == 0u);
                nextc[h] = group_code(w + U + h * kGroup);
            }
            if (dead) len = 0;
            if (len > 0) nsteps += min(U, w1 - w);
        }
        if constexpr (FIELDS) {
            const __amdgpu_buffer_rsrc_t re = buffer_rsrc(plane0 + off, len);
            const __amdgpu_buffer_rsrc_t ra = buffer_rsrc(plane1 + off, len);
#pragma unroll
            for (int q = 0; q < U; ++q) {
                st.e[q] = __builtin_bit_cast(v2f, __builtin_amdgcn_raw_buffer_load_b64(re, lane_ld,
                                                                                      (int)(q * step_bytes), 0));
                st.a[q] = __builtin_bit_cast(v2f, __builtin_amdgcn_raw_buffer_load_b64(ra, lane_ld,
                                                                                      (int)(q * step_bytes), 0));
            }
        } else if constexpr (MODE == MODE_VJP_GEPS) {
            const __amdgpu_buffer_rsrc_t rg = buffer_rsrc(plane0 + off, len);
#pragma unroll
            for (int q = 0; q < U; ++q)
                st.g[q] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rg, lane_off,
                                                                                        (int)(q * step_bytes), 0));
        }
        if constexpr (!SPARSE) {
#pragma unroll
            for (int h = 0; h < NG; ++h) st.gc[h] = group_code(w + h * kGroup);
        }
    };
    // the first two sets of U steps (every segment holds at least one step);
    // when they go out depends on the feature set (below)
    auto first_loads = [&]() {
        if constexpr (VJP && !SPARSE) {
            load_set(sa, w0);
            load_set(sb, w0 + U);
        }
    };

    // ---- 1. in-plane sums
    double F[NC], F2[NC];
    int ncand = 0;
    bool staged_all = false;
    bool live = true;    // sparse: some in-plane partial of the sample can be nonzero
    // F cache (eps_build, eps_grad_vjp, eps_grad_vjp_geps): when no field
    // has changed since the planes were written (chg[gen % 3] == 0, set by
    // the stage kernel), F comes from the planes and the prologue only lists
    // and stages the candidates (for the partials); otherwise the kernel
    // evaluates F and writes it there (and the fields it came from) for the
    // next call at the same p.
    // (not in the 8-class catch-all kernel, nor the catch-all backward of
    // eps_grad_vjp_geps: their registers do not hold both prologues)
    constexpr bool CACHE = (MODE == MODE_EPS || MODE == MODE_VJP_FIELDS || MODE == MODE_VJP_GEPS) &&
                           TREE != TR_GEN8 && !(MODE == MODE_VJP_GEPS && TREE == TR_GEN4);
    const int64_t nuv = (int64_t)P.nu * P.nv;
    const int64_t fidx = (int64_t)comp * P.nclass * nuv + (int64_t)G.uu + (int64_t)G.vv * P.nu;
    bool cached = false;
    if constexpr (CACHE) {
        if (P.fplane != nullptr)
            cached = __builtin_amdgcn_readfirstlane(*(volatile const int*)(P.chg + P.gen % 3)) == 0;
    }
    if (cached) {
#pragma unroll
        for (int c = 0; c < NC; ++c) F[c] = (c < P.nclass) ? P.fplane[fidx + (int64_t)c * nuv] : 0.0;
    }
    // feature sets that use the F cache: the first loads go out before the
    // staging only when F comes from the planes; an evaluating call issues them
    // after its FP64 in-plane sums, so the loads' registers are not live during
    // the evaluation (which lets the kernel fit one more wavefront per SIMD)
    constexpr bool CACHED_SET = (TYPES & (T_ELL | T_POLAR | T_SERIES)) != 0 && !SPARSE;
    if constexpr (VJP && CACHED_SET) {
        // ellipse set: a cached call's first loads go out before its list is
        // read and staged (grating coupler 122.9 -> 121.7 us; the Fourier
        // set measured about 1 us slower that way, and keeps them after)
        constexpr bool EARLY_LISTED = TYPES == (T_BOX | T_ELL);
        if (cached) {
            // the tile's candidates from the list the evaluating call kept (no scan)
            if constexpr (EARLY_LISTED) first_loads();
            bool listed = false;
            if (P.tlist != nullptr && !P.linear && __builtin_amdgcn_readfirstlane(P.tlist[0]) == P.tu) {
                const int32_t* tl = P.tlist + 1 + (int64_t)tile * (1 + kStageRec);
                const int cnt = __builtin_amdgcn_readfirstlane(tl[0]);
                if (cnt >= 0) {
                    if (tid < cnt) s_cand[tid] = tl[1 + tid];
                    stage_cands(P.prec, s_cand, 0, cnt, s_rec);     // barriers before and after
                    ncand = cnt;
                    staged_all = true;
                    listed = true;
                    if constexpr (!EARLY_LISTED) first_loads();
                }
            }
            if (!listed)
                inplane_sums<NC, TYPES, SIGS, SPARSE>(P, P.bbox, P.prec, P.fval, G.T, comp, G.uu, G.uc, G.uw, G.vc,
                                                      G.vw, s_cand, s_cnt, s_rec, F, ncand, staged_all,
                                                      [&] {
                                                          if constexpr (!EARLY_LISTED) first_loads();
                                                      },
                                                      &live, false);
        } else {
            inplane_sums<NC, TYPES, SIGS, SPARSE>(P, P.bbox, P.prec, P.fval, G.T, comp, G.uu, G.uc, G.uw, G.vc, G.vw,
                                                  s_cand, s_cnt, s_rec, F, ncand, staged_all, [] {}, &live, true);
            first_loads();
        }
    } else if constexpr (VJP) {
        // (the sets go out before the candidate scan: the stream's first
        // steps arrive while the tile's candidates are listed and staged;
        // measured on the taper, 132.6 -> 131.1 us)
        first_loads();
        inplane_sums<NC, TYPES, SIGS, SPARSE>(P, P.bbox, P.prec, P.fval, G.T, comp, G.uu, G.uc, G.uw, G.vc, G.vw,
                                              s_cand, s_cnt, s_rec, F, ncand, staged_all, [] {}, &live, !cached);
    } else if (!cached) {
        inplane_sums<NC, TYPES, SIGS, SPARSE>(P, P.bbox, P.prec, P.fval, G.T, comp, G.uu, G.uc, G.uw, G.vc, G.vw,
                                              s_cand, s_cnt, s_rec, F, ncand, staged_all, first_loads, &live);
    }
    if (!cached) {
        if constexpr (CACHE) {
            if (P.fplane != nullptr) {
                if (seg == 0 && act) {
#pragma unroll
                    for (int c = 0; c < NC; ++c)
                        if (c < P.nclass) P.fplane[fidx + (int64_t)c * nuv] = F[c];
                }
                for (int i = b * kBlock + tid; i < P.nfield; i += (int)gridDim.x * kBlock) P.fprev[i] = P.fval[i];
                if (P.tlist != nullptr) {
                    // the tile's candidates (s_cand holds them when they fit one staging round)
                    if (b == 0 && tid == 0) P.tlist[0] = P.linear ? -1 : P.tu;
                    if (!P.linear && seg == 0) {
                        int32_t* tl = P.tlist + 1 + (int64_t)tile * (1 + kStageRec);
                        if (tid == 0) tl[0] = staged_all ? ncand : -1;
                        if (staged_all && tid < ncand) tl[1 + tid] = s_cand[tid];
                    }
                }
            }
        }
    }
    if constexpr (FDM) {
        int nc2;
        bool sa2;
        inplane_sums<NC, TYPES, SIGS>(P, P.bbox2, P.prec2, P.fval2, G.T, comp, G.uu, G.uc, G.uw, G.vc, G.vw, s_cand,
                                      s_cnt, s_rec, F2, nc2, sa2, [] {});
    }

    // ---- 2. the column
    if constexpr (MODE == MODE_FD_SPARSE) {
        // sum over the column segment of g * deps (s(p + h) - s(p - h)), the
        // difference rounded to FP32 as the plane of MODE_FD stores it; g is
        // read kChunk steps at a time with every load of a chunk in flight
        constexpr int kChunk = 32;
        auto diff = [&](const double (&Z)[NC], const double (&Z2)[NC]) -> float {
            return (float)(P.deps * (compose<TREE>(P, F, Z).s - compose<TREE>(P, F2, Z2).s));
        };
        const char* gb = reinterpret_cast<const char*>(P.geps + (int64_t)comp * P.plane);
        const int64_t g_bytes = P.plane * 4;
        const int64_t g_step = P.sw * 4;
        const uint32_t g_lane = (uint32_t)b0 * 4;
        double acc = 0.0;
        uint32_t cur = 0xFFFFFFFFu;
        float run_out = 0.0f;
        for (int wc = w0; wc < w1; wc += kChunk) {
            const int64_t off = (int64_t)wc * g_step;
            const __amdgpu_buffer_rsrc_t rg = buffer_rsrc(gb + off, min(g_bytes - off, (int64_t)(w1 - wc) * g_step));
            float g[kChunk];
#pragma unroll
            for (int q = 0; q < kChunk; ++q)
                g[q] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rg, g_lane, (int)(q * g_step), 0));
#pragma unroll
            for (int q = 0; q < kChunk; ++q) {
                const int w = wc + q;
                if (w < w1) {
                    const uint32_t c = step_code(w);
                    float d;
                    if (c & kCodeGeneral) {
                        double Z[NC], Z2[NC];
                        load_zt(ztab, w, Z);
                        load_zt(ztab2, w, Z2);
                        d = diff(Z, Z2);
                    } else {
                        if (c != cur) {
                            double Z[NC], Z2[NC];
                            mask_z<NC>(c & 0xFFu, Z);
                            mask_z<NC>((c >> 8) & 0xFFu, Z2);
                            run_out = diff(Z, Z2);
                            cur = c;
                        }
                        d = run_out;
                    }
                    acc += (double)g[q] * (double)d;
                }
            }
        }
        if (!act) acc = 0.0;
        // block sum, one atomic per block
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
        __shared__ double s_fd[kBlock / 64];
        if ((tid & 63) == 0) s_fd[wave] = acc;
        __syncthreads();
        if (tid == 0) {
            double t = 0.0;
#pragma unroll
            for (int i = 0; i < kBlock / 64; ++i) t += s_fd[i];
            if (t != 0.0) atomicAdd(P.grad + P.fd_k, t * P.fd_scale);
        }
        return;
    } else if constexpr (MODE == MODE_EPS || MODE == MODE_FD) {
        auto value = [&](const double (&Z)[NC], const double (&Z2)[NC]) -> float {
            const double s = compose<TREE>(P, F, Z).s;
            if constexpr (MODE == MODE_EPS) {
                return (float)(P.eps_bg + P.deps * s);
            } else {
                const double s2 = compose<TREE>(P, F2, Z2).s;
                return (float)(P.deps * (s - s2));
            }
        };
        const char* outb = reinterpret_cast<const char*>(P.out + (int64_t)comp * P.plane);
        const int64_t out_bytes = P.plane * 4;
        const int64_t out_step = P.sw * 4;
        const uint32_t out_lane = (uint32_t)b0 * 4;
        uint32_t cur = 0xFFFFFFFFu;    // mask of the current run (none yet)
        float run_out = 0.0f;
        // scalar bookkeeping kept to a minimum (the scalar unit is shared by
        // the CU's wavefronts): the group's resource and the next group's code
        // advance incrementally, and a whole group's stores go out unguarded
        const int64_t gbytes = (int64_t)kGroup * out_step;
        const char* ob = outb + (int64_t)w0 * out_step;
        int64_t left = out_bytes - (int64_t)w0 * out_step;
        int gi = w0 / kGroup;          // segments start at a group boundary
        uint32_t gc_next = combine(gcode[gi], FDM ? gcode2[gi] : 0u);
        // eps_build with static codes: a run of full groups with one binary
        // code is one value and a loop of stores (one resource for the run,
        // the step offset in the scalar offset, the lanes' q offsets fixed)
        const ConstU32 grun = const_space<ConstU32>(P.grun != nullptr ? P.grun + (int64_t)comp * ngw : nullptr);
        const int gfull = w1 / kGroup;     // groups [w0 / kGroup, gfull) hold kGroup steps of the segment
        uint32_t vq[kGroup];
#pragma unroll
        for (int q = 0; q < kGroup; ++q) vq[q] = out_lane + (uint32_t)(q * out_step);
        for (int w = w0; w < w1; w += kGroup) {
            if constexpr (MODE == MODE_EPS) {
                const uint32_t gc = gc_next;
                if (P.grun != nullptr && !(gc & kCodeGeneral) && gi < gfull) {
                    // groups [gi, ge): code gc, all full; at most 2^31 bytes of offsets
                    const int64_t capg = ((int64_t)0x7FFFFFFF - 3 * out_step) / gbytes;
                    const int cap = (int)(capg < (1 << 20) ? capg : (1 << 20));
                    const int ge = min(min((int)grun[gi], gfull), gi + max(cap, 1));
                    if (gc != cur) {
                        double Z[NC];
                        mask_z<NC>(gc & 0xFFu, Z);
                        run_out = value(Z, Z);
                        cur = gc;
                    }
                    if (act) {
                        const __amdgpu_buffer_rsrc_t rr = buffer_rsrc(ob, (int64_t)(ge - gi) * gbytes);
                        uint32_t so = 0;
                        for (int g = gi; g < ge; ++g) {
#pragma unroll
                            for (int q = 0; q < kGroup; ++q)
                                __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, run_out), rr,
                                                                      vq[q], (int)so, 2);
                            so += (uint32_t)gbytes;
                        }
                    }
                    ob += (int64_t)(ge - gi) * gbytes;
                    left -= (int64_t)(ge - gi) * gbytes;
                    w = (ge - 1) * kGroup;          // the loop adds kGroup
                    gi = min(ge, ngw - 1);
                    gc_next = gcode[gi];
                    continue;
                }
            }
            const __amdgpu_buffer_rsrc_t ro = buffer_rsrc(ob, left);
            const uint32_t gc = gc_next;
            gi = min(gi + 1, ngw - 1);
            gc_next = combine(gcode[gi], FDM ? gcode2[gi] : 0u);
            ob += gbytes;
            left -= gbytes;
            float out[kGroup];
            if (!(gc & kCodeGeneral) && w + kGroup <= w1) {
                if (gc != cur) {
                    double Z[NC], Z2[NC];
                    mask_z<NC>(gc & 0xFFu, Z);
                    if constexpr (FDM) mask_z<NC>((gc >> 8) & 0xFFu, Z2);
                    run_out = value(Z, Z2);
                    cur = gc;
                }
#pragma unroll
                for (int q = 0; q < kGroup; ++q) out[q] = run_out;
            } else {
#pragma unroll
                for (int q = 0; q < kGroup; ++q) {
                    out[q] = 0.0f;
                    if (w + q < w1) {
                        const uint32_t c = step_code(w + q);
                        if (c & kCodeGeneral) {
                            double Z[NC], Z2[NC];
                            load_zt(ztab, w + q, Z);
                            if constexpr (FDM) load_zt(ztab2, w + q, Z2);
                            out[q] = value(Z, Z2);
                        } else {
                            if (c != cur) {
                                double Z[NC], Z2[NC];
                                mask_z<NC>(c & 0xFFu, Z);
                                if constexpr (FDM) mask_z<NC>((c >> 8) & 0xFFu, Z2);
                                run_out = value(Z, Z2);
                                cur = c;
                            }
                            out[q] = run_out;
                        }
                    }
                }
            }
            if (act) {
                // eps goes out non-temporal (the nt bit of the buffer store):
                // its lines leave the caches at once instead of being written
                // back while the next kernel streams its own inputs
                constexpr int kStorePolicy = (MODE == MODE_EPS) ? 2 : 0;
                if (w + kGroup <= w1) {
#pragma unroll
                    for (int q = 0; q < kGroup; ++q)
                        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, out[q]), ro, out_lane,
                                                              (int)(q * out_step), kStorePolicy);
                } else {
#pragma unroll
                    for (int q = 0; q < kGroup; ++q)
                        if (w + q < w1)
                            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, out[q]), ro, out_lane,
                                                                  (int)(q * out_step), kStorePolicy);
                }
            }
        }
        return;
    } else {
        float A[NC], Blo[NC], Bhi[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) A[c] = Blo[c] = Bhi[c] = 0.0f;
        // g of one step times gscale is d F / d eps at that sample, times deps
        const float gscale = (FIELDS ? P.two_omega : 1.0f) * (float)P.deps;
        // A_c += gd * cf_c * Z_c (and the w-bound partials on general steps)
        auto accumulate = [&](const Comp<NC>& o, const double (&Z)[NC], float gd, int w, bool general) {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                if (c < P.nclass) {
                    const float cc = gd * (float)o.cf[c];
                    A[c] += cc * (float)Z[c];
                    if (general && P.cls_wparam[c]) {
                        const int64_t zi = 3 * ((int64_t)c * P.nw + w);
                        Blo[c] += cc * (float)ztab[zi + 1];
                        Bhi[c] += cc * (float)ztab[zi + 2];
                    }
                }
            }
        };
        uint32_t cur = 0;     // mask of the current run of binary steps
        float grun = 0.0f;    // sum of g over that run
        auto flush = [&]() {
            if (cur != 0u) {
                double Z[NC];
                mask_z<NC>(cur, Z);
                accumulate(compose<TREE>(P, F, Z), Z, grun * gscale, 0, false);
            }
            grun = 0.0f;
        };
        auto process = [&](const Set& st, int w) {
#pragma unroll
            for (int h = 0; h < NG; ++h) {
                const int wg = w + h * kGroup;
                if (wg >= w1) break;
                float g[kGroup];
#pragma unroll
                for (int q = 0; q < kGroup; ++q) {
                    const int i = h * kGroup + q;
                    if constexpr (FIELDS)
                        g[q] = st.e[i].x * st.a[i].y + st.e[i].y * st.a[i].x;   // Im(E Eadj)
                    else
                        g[q] = st.g[i];
                }
                const uint32_t gc = st.gc[h];
                if (!(gc & kCodeGeneral) && wg + kGroup <= w1) {
                    if (gc != cur) {
                        flush();
                        cur = gc;
                    }
                    grun += (g[0] + g[1]) + (g[2] + g[3]);
                } else {
#pragma unroll
                    for (int q = 0; q < kGroup; ++q) {
                        if (wg + q < w1) {
                            const uint32_t c = step_code(wg + q);
                            if (c & kCodeGeneral) {
                                double Z[NC];
                                load_zt(ztab, wg + q, Z);
                                accumulate(compose<TREE>(P, F, Z), Z, g[q] * gscale, wg + q, true);
                            } else {
                                if (c != cur) {
                                    flush();
                                    cur = c;
                                }
                                grun += g[q];
                            }
                        }
                    }
                }
            }
        };
        // The loads are issued unconditionally (reads past the plane return
        // 0): a load under a branch makes the wait before the next set drain
        // every outstanding load, which turns the double buffer back into
        // load-wait-compute.
        bool stream = true;
        uint64_t lm = 0;    // sparse: live lanes of the wavefront
        if constexpr (SPARSE) {
            // columns with column-axis parameters feed their bound partials
            // wherever F_c is nonzero: every sample is read then
            bool wpar = false;
#pragma unroll
            for (int c = 0; c < NC; ++c) wpar = wpar || (c < P.nclass && P.cls_wparam[c]);
            live = act && (live || wpar);
            lm = __ballot(live);
            stream = lm != 0;
            if (stream) {
                const int lead = uniform_int(__ffsll((unsigned long long)lm) - 1);
                const uint32_t lead_off = (uint32_t)__builtin_amdgcn_readlane((int)lane_off, lead);
                lane_ld = live ? lane_off : lead_off;
#pragma unroll
                for (int h = 0; h < NG; ++h) nextc[h] = group_code(w0 + h * kGroup);
                load_set(sa, w0);
                load_set(sb, w0 + U);
            }
        }
        if (stream) {
            const int nset = (w1 - w0 + U - 1) / U;
            for (int si = 0; si < nset; si += 2) {
                process(sa, w0 + si * U);
                load_set(sa, w0 + (si + 2) * U);
                process(sb, w0 + (si + 1) * U);
                load_set(sb, w0 + (si + 3) * U);
            }
            flush();
        }
        if constexpr (SPARSE) {
            // spread over kReadSlots counters: one address taking an atomic
            // from every wavefront of the grid serializes them
            if (P.nread != nullptr && (tid & 63) == 0 && nsteps > 0)
                atomicAdd(P.nread + ((blockIdx.x * (kBlock / 64) + wave) & (kReadSlots - 1)),
                          (unsigned long long)__popcll(lm) * (unsigned long long)nsteps);
            // nothing to add from a block with no live sample
            if (!__syncthreads_or(live ? 1 : 0)) return;
        }

        // ---- 3. partials of the column-axis bounds of each class (F_c times
        // the w-bound sums), then the in-plane partials
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if (c < P.nclass && P.cls_wparam[c]) {
                const DevClass cl = P.cls[c];
                const float fs = act ? (float)F[c] : 0.0f;
                emit(P, cl.flo, fs * Blo[c]);
                emit(P, cl.fhi, fs * Bhi[c]);
            }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) sA[c * kBlock + tid] = (act && live) ? A[c] : 0.0f;
        s_lat[tid] = G.uc;
        s_lat[kBlock + tid] = G.uw;
        s_lat[2 * kBlock + tid] = G.vc;
        s_lat[3 * kBlock + tid] = G.vw;
        const SampleLat L{s_lat};
        float* sgw = sG + ((TYPES & T_GCART) ? wave * 2 * kSegBucket : 0);
        const int u0 = G.u - (tid & (P.tu - 1));   // first u of the tile
        if constexpr ((TYPES & T_POLAR) != 0) {
            // coefficient slots: unclaimed (the barrier below, or the scan's, orders this before use)
            if (tid < kPolarSlots) {
                s_pkey[tid] = -2;
                s_pacc[tid] = 0.0;
            }
        }
        PolarAcc pacc;
        polar_acc_clear(pacc);
        if (staged_all) {
            __syncthreads();
            for (int j = wave; j < ncand; j += kBlock / 64)
                block_partials<TYPES, SIGS>(P, s_rec[j], sA + s_rec[j].pr.cls * kBlock, L, G.T, comp, u0, sgw,
                                            s_pacc, s_pkey, pacc);
            series_split<TYPES, SIGS>(P, s_rec, ncand, sA, L);
        } else {
            for (int next = 0; next < P.nprim;) {
                const int n = scan_candidates(P.bbox, P.nprim, next, G.T.ulo, G.T.uhi, G.T.vlo, G.T.vhi, s_cand,
                                              s_cnt, &next);
                for (int j0 = 0; j0 < n; j0 += kStageRec) {
                    const int nj = min(kStageRec, n - j0);
                    stage_cands(P.prec, s_cand, j0, nj, s_rec);
                    for (int j = wave; j < nj; j += kBlock / 64)
                        block_partials<TYPES, SIGS>(P, s_rec[j], sA + s_rec[j].pr.cls * kBlock, L, G.T, comp, u0,
                                                    sgw, s_pacc, s_pkey, pacc);
                    series_split<TYPES, SIGS>(P, s_rec, nj, sA, L);
                }
            }
        }
        if constexpr ((TYPES & T_POLAR) != 0) {
            polar_acc_flush(P, pacc, s_pacc, s_pkey);
            // one atomic per combined coefficient parameter
            __syncthreads();
            if (tid < kPolarSlots && s_pkey[tid] >= 0 && s_pacc[tid] != 0.0)
                atomicAdd(grad_copy(P) + s_pkey[tid], s_pacc[tid]);
        }
    }
}

// minimum wavefronts per SIMD the register allocation must leave room for:
// the box + sine-series variant sits 2 VGPRs over the 3-wave budget otherwise
template <int MODE, int TYPES>
constexpr int column_min_waves() {
    return (MODE == MODE_VJP_FIELDS && TYPES == (T_BOX | T_SERIES)) ? 3 : 1;
}

template <int MODE, int TREE, int TYPES, int SIGS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(column_min_waves<MODE, TYPES>())))
void k_column(const KParams P) {
    column_body<MODE, TREE, TYPES, SIGS>(P, blockIdx.x);
}

// Several requests in one launch: request r owns blocks [first[r], first[r+1])
// and its own parameter block plist[r] (same kernel specialization); they are
// its blocks plist[r].block0 + [0, first[r+1] - first[r]).
template <int MODE, int TREE, int TYPES, int SIGS>
__global__ __launch_bounds__(256) void k_column_batch(const KParams* __restrict__ plist,
                                                      const int* __restrict__ first, int nreq) {
    int lo = 0, hi = nreq;                   // first[lo] <= blockIdx.x < first[hi]
    const int b = blockIdx.x;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (first[mid] <= b) lo = mid; else hi = mid;
    }
    column_body<MODE, TREE, TYPES, SIGS>(plist[lo], b - first[lo] + plist[lo].block0);
}

// ------------------------------------------------------------------ launch templates
template <int MODE, int TYPES, int SIGS>
static hipError_t launch_variant(int tree, const KParams& kp, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    const int64_t blocks = (int64_t)kp.ncomp * kp.tiles_u * kp.tiles_v * kp.nseg;
    const dim3 grid((unsigned)blocks), blk(256);
    // e0 / e1 (optional) take the kernel's own start and end times
    auto go = [&](auto kern) { hipExtLaunchKernelGGL(kern, grid, blk, 0, st, e0, e1, 0, kp); };
    switch (tree) {
        case TR_U1: go(k_column<MODE, TR_U1, TYPES, SIGS>); break;
        case TR_U2: go(k_column<MODE, TR_U2, TYPES, SIGS>); break;
        case TR_D11: go(k_column<MODE, TR_D11, TYPES, SIGS>); break;
        case TR_D12: go(k_column<MODE, TR_D12, TYPES, SIGS>); break;
        default:
            // generic op trees only come with the catch-all feature set
            if constexpr (TYPES == T_ALL && SIGS == S_ALL) {
                if (tree == TR_GEN4) go(k_column<MODE, TR_GEN4, TYPES, SIGS>);
                else go(k_column<MODE, TR_GEN8, TYPES, SIGS>);
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

template <int MODE>
hipError_t launch_mode(int tree, int variant, const KParams& kp, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    switch (variant) {
        case VAR_BOX_LIN: return launch_variant<MODE, T_BOX, S_LIN>(tree, kp, st, e0, e1);
        case VAR_GCART_LIN: return launch_variant<MODE, T_BOX | T_GCART, S_LIN>(tree, kp, st, e0, e1);
        case VAR_ELL_SIGMOID: return launch_variant<MODE, T_BOX | T_ELL, S_LIN | S_SIGMOID>(tree, kp, st, e0, e1);
        case VAR_POLAR_SIGMOID: return launch_variant<MODE, T_BOX | T_POLAR, S_LIN | S_SIGMOID>(tree, kp, st, e0, e1);
        case VAR_SERIES_LIN: return launch_variant<MODE, T_BOX | T_SERIES, S_LIN>(tree, kp, st, e0, e1);
        default: return launch_variant<MODE, T_ALL, S_ALL>(tree, kp, st, e0, e1);
    }
}

// launch_mode is instantiated once per mode, in its own translation unit
extern template hipError_t launch_mode<MODE_EPS>(int, int, const KParams&, hipStream_t, hipEvent_t, hipEvent_t);
extern template hipError_t launch_mode<MODE_VJP_FIELDS>(int, int, const KParams&, hipStream_t, hipEvent_t, hipEvent_t);
extern template hipError_t launch_mode<MODE_VJP_GEPS>(int, int, const KParams&, hipStream_t, hipEvent_t, hipEvent_t);
extern template hipError_t launch_mode<MODE_FD>(int, int, const KParams&, hipStream_t, hipEvent_t, hipEvent_t);
extern template hipError_t launch_mode<MODE_VJP_SPARSE>(int, int, const KParams&, hipStream_t, hipEvent_t, hipEvent_t);
extern template hipError_t launch_mode<MODE_FD_SPARSE>(int, int, const KParams&, hipStream_t, hipEvent_t, hipEvent_t);

}  // namespace sg

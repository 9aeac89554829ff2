// gfx950 kernels of the shape-gradient path outside the column kernel, and
// the launch dispatch.
//
//  k_stage   p -> resolved primitive fields (a + b p[idx]), support boxes,
//            per-primitive records, the per-class extrusion tables Z(w),
//            dZ/dlo, dZ/dhi and the column-step codes; zeroes the gradient
//            accumulator.
//  k_gplane  g = 2 omega Im(E Eadj) plane (finite-difference baseline)
//  k_dot     sum a * b (finite-difference baseline reduction)
// The column kernel (sg_column.h) is compiled per mode in sg_mode_*.hip.
#include "sg_column.h"

namespace sg {

// ------------------------------------------------------------------ stage
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Blocks [0, prim_blocks) take one primitive per wavefront: its fields are
// resolved by the lanes in parallel, the support box is reduced across the
// wavefront and lane 0 writes the primitive's record.  The remaining blocks
// take one (component, group of column steps) or one gradient entry per thread.
__global__ __launch_bounds__(256) void k_stage(const StageParams sp) {
    const int var = blockIdx.y;
    const double delta = sp.delta[var];
    auto resolve = [&](int f) -> double {
        const sg_field r = sp.fref[f];
        if (r.idx < 0) return r.a;
        double pv = sp.p[r.idx];
        if (r.idx == sp.pert_idx) pv += delta;
        return r.a + r.b * pv;
    };
    const int prim_blocks = (sp.nprim + 3) / 4;
    if (sp.fprev != nullptr && var == 0 && blockIdx.x == 0 && threadIdx.x == 0) {
        sp.chg[(sp.gen + 1) % 3] = 0;
        if (sp.force) sp.chg[sp.gen % 3] = 1;
    }
    if ((int)blockIdx.x < prim_blocks) {
        const int lane = threadIdx.x & 63;
        const int pi = (int)blockIdx.x * 4 + (int)(threadIdx.x >> 6);
        if (pi >= sp.nprim) return;
        const DevPrim pr = sp.prims[pi];
        double* fv = sp.fval[var];
        int nf;
        switch (pr.type) {
            case SG_PRIM_BOX: nf = 6; break;
            case SG_PRIM_ELLIPSE: nf = 5; break;
            case SG_PRIM_POLY: nf = 2 * pr.nvert + 2; break;
            case SG_PRIM_POLAR: nf = 2 * pr.nvert + 5; break;
            case SG_PRIM_POLAR2D: nf = 6; break;
            case SG_PRIM_SERIES: nf = pr.nvert + 4; break;
            default: nf = 2 * pr.nvert + 4; break;
        }
        // lane i resolves fields f0 + i, f0 + i + 64, ...; the first one stays
        // in the lane for the boxes' and ellipses' record fields.  Each round
        // of kStageUnroll fields per lane issues all its loads (references,
        // previous fields, then parameters) before any store: the stores to
        // fval may alias the inputs as far as the compiler knows, so a
        // load-store-load loop would wait out one memory latency per field.
        constexpr int kStageUnroll = 4;
        double v0 = 0.0, b0 = 0.0;
        double vabs = 0.0;    // SERIES: sum of |v_i| over this lane's sine coefficients
        double ylo = __builtin_huge_val(), yhi = -__builtin_huge_val();   // GCART: extent of y+ and y-
        int idx0 = -1;
        bool changed = false;
        const bool cmp = sp.fprev != nullptr && var == 0;
        for (int base = 0; base < nf; base += 64 * kStageUnroll) {
            sg_field r[kStageUnroll];
            double prev[kStageUnroll], pv[kStageUnroll];
#pragma unroll
            for (int k = 0; k < kStageUnroll; ++k) {
                const int i = base + k * 64 + lane;
                r[k] = (i < nf) ? sp.fref[pr.f0 + i] : sg_field{0.0, 0.0, -1};
                prev[k] = (cmp && i < nf) ? sp.fprev[pr.f0 + i] : 0.0;
            }
#pragma unroll
            for (int k = 0; k < kStageUnroll; ++k) {
                pv[k] = (r[k].idx >= 0) ? sp.p[r[k].idx] : 0.0;
                if (r[k].idx >= 0 && r[k].idx == sp.pert_idx) pv[k] += delta;
            }
#pragma unroll
            for (int k = 0; k < kStageUnroll; ++k) {
                const int i = base + k * 64 + lane;
                if (i >= nf) break;
                const double v = (r[k].idx >= 0) ? r[k].a + r[k].b * pv[k] : r[k].a;
                fv[pr.f0 + i] = v;
                // bitwise comparison (a NaN field always counts as changed)
                if (cmp && __double_as_longlong(prev[k]) != __double_as_longlong(v)) changed = true;
                if (i >= 2 && i < 2 + pr.nvert) {
                    vabs += fabs(v);
                    yhi = fmax(yhi, v);
                } else if (i >= 2 + pr.nvert && i < 2 + 2 * pr.nvert) {
                    ylo = fmin(ylo, v);
                }
                if (i == lane) {
                    v0 = v;
                    idx0 = r[k].idx;
                    b0 = r[k].b;
                }
            }
        }
        // a plain store (every writer writes 1): an atomic from each of
        // thousands of primitives to one address serializes
        if (__ballot(changed) != 0 && lane == 0) sp.chg[sp.gen % 3] = 1;
        const double inf = __builtin_huge_val();
        double4 b = make_double4(-inf, inf, -inf, inf);
        // lanes 0-3 fetch field f0 + koff: a box's u0 u1 v0 v1, otherwise the
        // first four fields (ellipse x0 y0 r; boundary x-range)
        int koff = min(lane, 3);
        if (pr.type == SG_PRIM_BOX) koff = (lane == 0 ? pr.fu0 : lane == 1 ? pr.fu1 : lane == 2 ? pr.fv0 : pr.fv1) - pr.f0;
        const double kv = __shfl(v0, koff, 64);
        const int kidx = __shfl(idx0, koff, 64);
        const double kb = __shfl(b0, koff, 64);
        const double r0 = __shfl(kv, 0, 64), r1 = __shfl(kv, 1, 64), r2 = __shfl(kv, 2, 64), r3 = __shfl(kv, 3, 64);
        if (pr.type == SG_PRIM_BOX) {
            if (pr.ubnd) { b.x = r0 - pr.reach0; b.y = r1 + pr.reach0; }
            if (pr.vbnd) { b.z = r2 - pr.reach1; b.w = r3 + pr.reach1; }
        } else if (pr.type == SG_PRIM_ELLIPSE) {
            const double R = r2 + pr.reach0;
            if (R < 0.0) b = make_double4(inf, -inf, inf, -inf);
            else b = make_double4(r0 - R * pr.ax, r0 + R * pr.ax, r1 - R * pr.ay, r1 + R * pr.ay);
        } else if (pr.type == SG_PRIM_POLY) {
            // the support is the polygon offset outward by reach0: its vertices
            // are v_i - d (n_{i-1} + n_i) / (1 + n_{i-1} . n_i), n inward normals
            auto resolve_f = [&](int f) -> double { return resolve(f); };
            const int N = pr.nvert;
            double xlo = inf, xhi = -inf, ylo = inf, yhi = -inf;
            bool open = false;
            for (int i = lane; i < N; i += 64) {
                const int ip = (i == 0) ? N - 1 : i - 1, in = (i + 1 == N) ? 0 : i + 1;
                const double xi = resolve_f(pr.f0 + i), yi = resolve_f(pr.f0 + N + i);
                const double xp = resolve_f(pr.f0 + ip), yp = resolve_f(pr.f0 + N + ip);
                const double xn = resolve_f(pr.f0 + in), yn = resolve_f(pr.f0 + N + in);
                const double ax = xi - xp, ay = yi - yp, bx = xn - xi, by = yn - yi;
                const double la = sqrt(ax * ax + ay * ay), lb = sqrt(bx * bx + by * by);
                const double nax = -ay / la, nay = ax / la, nbx = -by / lb, nby = bx / lb;
                const double den = 1.0 + nax * nbx + nay * nby;
                if (den > 1e-12) {
                    const double ox = xi - pr.reach0 * (nax + nbx) / den;
                    const double oy = yi - pr.reach0 * (nay + nby) / den;
                    xlo = fmin(xlo, ox); xhi = fmax(xhi, ox);
                    ylo = fmin(ylo, oy); yhi = fmax(yhi, oy);
                } else {
                    open = true;
                }
            }
            if (__ballot(open) != 0) b = make_double4(-inf, inf, -inf, inf);
            else b = make_double4(wave_min(xlo), wave_max(xhi), wave_min(ylo), wave_max(yhi));
        } else if (pr.type == SG_PRIM_SERIES) {
            // |f| <= the larger end of the linear ramp over [xs, xe] + sum |v_i| (envelope <= 1)
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) vabs += __shfl_xor(vabs, o, 64);
            const double* c = sp.consts + pr.c0;
            const double ra = fabs(0.5 * c[2] + 0.5 * (c[3] - c[2]) * (r0 - c[0]) / c[1]);
            const double rb = fabs(0.5 * c[2] + 0.5 * (c[3] - c[2]) * (r1 - c[0]) / c[1]);
            const double R = fmax(ra, rb) + vabs + pr.reach1;
            b = make_double4(r0 - pr.reach0, r1 + pr.reach0, c[4] - R, c[4] + R);
        } else if (pr.type == SG_PRIM_POLAR2D) {
            // |R (1 + delta cos)| <= |R| (1 + |delta|): a square about the center
            const double R = fabs(r2) * (1.0 + fabs(r3)) + pr.reach0;
            b = make_double4(r0 - R, r0 + R, r1 - R, r1 + R);
        } else if (pr.type == SG_PRIM_POLAR) {
            // R(theta) <= R0 + sum_n |c_n| + |s_n|: a square about the center
            double av = (lane >= 3 && lane < 3 + 2 * pr.nvert) ? fabs(v0) : 0.0;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) av += __shfl_xor(av, o, 64);
            const double R = fmax(r2 + av, 0.0) + pr.reach0;
            b = make_double4(r0 - R, r0 + R, r1 - R, r1 + R);
        } else {  // GCART: y+ are fields 2 .. M + 1, y- fields M + 2 .. 2 M + 1 (resolved above)
            const double ymax = wave_max(yhi), ymin = wave_min(ylo);
            b = make_double4(r0 - pr.reach0, r1 + pr.reach0, ymin - pr.reach1, ymax + pr.reach1);
        }
        // the record, written by the lanes together: the primitive's dwords,
        // then the support box and the four record fields
        PrimRec* rec = sp.prec[var] + pi;
        constexpr int kPrimDw = (int)(sizeof(DevPrim) / 4);
        if (lane < kPrimDw)
            reinterpret_cast<uint32_t*>(&rec->pr)[lane] = reinterpret_cast<const uint32_t*>(sp.prims + pi)[lane];
        if (lane < 4) {
            // boxes u0 u1 v0 v1, ellipses x0 y0 r, Fourier radius x0 y0 R0, Polar2D x0 y0 R delta
            const bool rf = pr.type == SG_PRIM_BOX || pr.type == SG_PRIM_ELLIPSE || pr.type == SG_PRIM_POLAR ||
                            pr.type == SG_PRIM_POLAR2D;
            const bool live = rf && (pr.type == SG_PRIM_BOX || pr.type == SG_PRIM_POLAR2D || lane < 3);
            rec->f[lane] = live ? kv : 0.0;
            rec->fb[lane] = live ? kb : 0.0;
            rec->fidx[lane] = live ? kidx : -1;
            const double bl = lane == 0 ? b.x : lane == 1 ? b.y : lane == 2 ? b.z : b.w;
            (&rec->bb.x)[lane] = bl;
        }
        if (lane == 0) {
            // outward rounding keeps the FP32 box a superset of the support
            sp.bbox[var][pi] = make_float4(__double2float_rd(b.x), __double2float_ru(b.y), __double2float_rd(b.z),
                                           __double2float_ru(b.w));
        }
        return;
    }
    const int64_t t = (int64_t)(blockIdx.x - prim_blocks) * blockDim.x + threadIdx.x;
    if (var == 0 && sp.zero_ptr != nullptr && t < sp.zero_n) sp.zero_ptr[t] = 0.0;
    // extrusion tables, step codes and group codes: one thread per
    // (component, group of kGroup column steps)
    const int ngw = (sp.nw + kGroup - 1) / kGroup;
    if (sp.tables && t < (int64_t)sp.ncomp * ngw) {
        const int g = (int)(t % ngw);
        const int comp = (int)(t / ngw);
        const int wb = g * kGroup;
        const int nq = min(kGroup, sp.nw - wb);
        double wc[kGroup], ww[kGroup];
#pragma unroll
        for (int q = 0; q < kGroup; ++q) {
            wc[q] = sp.wc[comp][wb + min(q, nq - 1)];
            ww[q] = sp.ww[comp][wb + min(q, nq - 1)];
        }
        uint32_t mask[kGroup] = {0, 0, 0, 0};
        bool binary[kGroup] = {true, true, true, true};
        // every class's bounds resolved before the first table store (one
        // chain of loads, not one per class)
        double clo[kMaxClasses], chi[kMaxClasses];
        bool cwp[kMaxClasses];
#pragma unroll
        for (int c = 0; c < kMaxClasses; ++c) {
            clo[c] = chi[c] = 0.0;
            cwp[c] = false;
            if (c < sp.nclass && sp.cls[c].bounded) {
                clo[c] = resolve(sp.cls[c].flo);
                chi[c] = resolve(sp.cls[c].fhi);
                cwp[c] = sp.fref[sp.cls[c].flo].idx >= 0 || sp.fref[sp.cls[c].fhi].idx >= 0;
            }
        }
        for (int c = 0; c < sp.nclass; ++c) {
            const DevClass cl = sp.cls[c];
            double lo = 0.0, hi = 0.0;
            bool wparam = false;
#pragma unroll
            for (int k = 0; k < kMaxClasses; ++k)
                if (k == c) {
                    lo = clo[k];
                    hi = chi[k];
                    wparam = cwp[k];
                }
            double* zt = sp.ztab[var] + 3 * (((int64_t)comp * sp.nclass + c) * sp.nw + wb);
#pragma unroll
            for (int q = 0; q < kGroup; ++q) {
                if (q >= nq) break;
                double z = 1.0, dlo = 0.0, dhi = 0.0;
                if (cl.bounded) rect_vd<S_ALL>(cl.skind, kval(cl.smode, cl.k, ww[q]), wc[q], lo, hi, z, dlo, dhi);
                zt[3 * q] = z;
                zt[3 * q + 1] = dlo;
                zt[3 * q + 2] = dhi;
                if (z == 1.0) mask[q] |= 1u << c;
                else if (z != 0.0) binary[q] = false;
                if (wparam && (dlo != 0.0 || dhi != 0.0)) binary[q] = false;
            }
        }
        uint32_t gcode = 0;
#pragma unroll
        for (int q = 0; q < kGroup; ++q) {
            if (q >= nq) break;
            const uint32_t code = binary[q] ? mask[q] : kCodeGeneral;
            sp.code[var][(int64_t)comp * sp.nw + wb + q] = code;
            if (q == 0) gcode = code;
            else if (code != gcode) gcode = kCodeGeneral;
        }
        sp.gcode[var][t] = gcode;
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
// Elements [i0, i1) only (a served request draws its planes in slices).
__global__ __launch_bounds__(256) void k_fieldgen(float2* __restrict__ e, float2* __restrict__ a, int64_t i0,
                                                  int64_t i1, uint32_t k0, uint32_t k1) {
    const float scale = 2.3283064365386963e-10f;   // 2^-32
    for (int64_t i = i0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < i1; i += (int64_t)gridDim.x * blockDim.x) {
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
    const int64_t nz = sp.tables ? (int64_t)sp.ncomp * ((sp.nw + kGroup - 1) / kGroup) : 0;
    const int64_t n = std::max<int64_t>(1, std::max<int64_t>(nz, sp.zero_n));
    const int64_t blocks = (sp.nprim + 3) / 4 + (n + 255) / 256;
    hipLaunchKernelGGL(k_stage, dim3((unsigned)blocks, (unsigned)nvariant), dim3(256), 0, st, sp);
    return hipGetLastError();
}

hipError_t launch_column(int mode, int tree, int variant, const KParams& kp, hipStream_t st, hipEvent_t e0,
                         hipEvent_t e1) {
    switch (mode) {
        case MODE_EPS: return launch_mode<MODE_EPS>(tree, variant, kp, st, e0, e1);
        case MODE_VJP_FIELDS: return launch_mode<MODE_VJP_FIELDS>(tree, variant, kp, st, e0, e1);
        case MODE_VJP_GEPS: return launch_mode<MODE_VJP_GEPS>(tree, variant, kp, st, e0, e1);
        case MODE_VJP_SPARSE: return launch_mode<MODE_VJP_SPARSE>(tree, variant, kp, st, e0, e1);
        case MODE_FD_SPARSE: return launch_mode<MODE_FD_SPARSE>(tree, variant, kp, st, e0, e1);
        default: return launch_mode<MODE_FD>(tree, variant, kp, st, e0, e1);
    }
}

// grad[k] from the fixed-point accumulators fx[3k .. 3k + 2] (fraction bits
// 0..31, fraction bits 32..63, integer part): the value is
// (a2 2^64 + a1 2^32 + a0) 2^-64, carried into a signed 64-bit integer part
// and a 64-bit fraction before the one conversion to FP64.  A range flag set
// by any addition makes every entry NaN.
__global__ __launch_bounds__(256) void k_fx_finish(const unsigned long long* __restrict__ fx, int64_t n,
                                                   double* __restrict__ grad) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    if (fx[3 * n] != 0ull) {
        grad[k] = __builtin_nan("");
        return;
    }
    const unsigned long long a0 = fx[3 * k], a1 = fx[3 * k + 1], a2 = fx[3 * k + 2];
    const unsigned long long lo = a0 + (a1 << 32);
    const long long hi = (long long)(a2 + (a1 >> 32) + (lo < a0 ? 1ull : 0ull));
    grad[k] = (double)hi + (double)lo * 0x1p-64;
}

// grad[k] = sum of the kGradSpread copies, in copy order.
__global__ __launch_bounds__(256) void k_spread_finish(const double* __restrict__ sp, int64_t n,
                                                       double* __restrict__ grad) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double s = 0.0;
#pragma unroll 8
    for (int c = 0; c < kGradSpread; ++c) s += sp[c * n + k];
    grad[k] = s;
}

hipError_t launch_spread_finish(const double* spread, int64_t n, double* grad, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_spread_finish, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, spread, n, grad);
    return hipGetLastError();
}

hipError_t launch_fx_finish(const unsigned long long* fx, int64_t n, double* grad, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fx_finish, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, fx, n, grad);
    return hipGetLastError();
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

hipError_t launch_fieldgen(float2* e, float2* a, int64_t i0, int64_t i1, uint64_t seed, hipStream_t st) {
    const int64_t blocks = std::min<int64_t>(8192, (i1 - i0 + 255) / 256);
    hipLaunchKernelGGL(k_fieldgen, dim3((unsigned)std::max<int64_t>(1, blocks)), dim3(256), 0, st, e, a, i0, i1,
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

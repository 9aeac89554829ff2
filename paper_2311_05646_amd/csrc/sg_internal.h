// Internal tables shared by the host scene compiler and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/shapegrad.h"

namespace sg {

constexpr int kMaxComp = 3;
constexpr int kMaxClasses = 8;
constexpr int kMaxNodes = 6;       // op-tree nodes of the general composition program
constexpr int kBlock = 256;        // threads (= in-plane samples) per block
// copies of the gradient that blocks spread their FP64 atomics over when a
// parameter is shared by many blocks (one address taking an atomic from every
// block serializes them)
constexpr int kGradSpread = 32;
constexpr int kCandCap = 2048;     // candidate primitives listed in LDS per pass
constexpr int kStageRec = 32;      // candidate records staged in LDS per round
constexpr int kZStage = 512;       // extrusion-table entries staged in LDS per chunk
constexpr int kReadSlots = 256;    // partial counters of the sparse VJP's read statistic

// MODE_VJP_SPARSE: the fused VJP reading only the samples whose in-plane
// derivatives do not all vanish and the column steps with a class at nonzero
// extrusion (same result as MODE_VJP_FIELDS up to summation order).
// MODE_FD_SPARSE: one parameter's central / forward difference restricted to
// the tiles its primitives' support boxes meet (at either evaluation point)
// and to the steps where a class is nonzero, multiplied by the g plane and
// reduced in the same pass (no difference plane).
enum Mode { MODE_EPS = 0, MODE_VJP_FIELDS = 1, MODE_VJP_GEPS = 2, MODE_FD = 3, MODE_VJP_SPARSE = 4, MODE_FD_SPARSE = 5 };
// Column-step codes written by k_stage, one per (component, w): bits 0-7 hold
// the mask of classes whose extrusion factor is exactly 1 when every class
// factor is exactly 0 or 1 (and the w-bound derivatives of classes with
// column-axis parameters vanish); kCodeGeneral marks any other step.  A group
// code covers kGroup consecutive steps starting at a multiple of kGroup: their
// common code, or kCodeGeneral when they differ.
constexpr uint32_t kCodeGeneral = 1u << 16;
constexpr int kGroup = 4;    // the stage kernel and the stream kernel's group paths assume 4
// kernel feature variants (primitive types x in-plane sigma kinds), smallest first
enum Variant { VAR_BOX_LIN = 0, VAR_GCART_LIN = 1, VAR_ELL_SIGMOID = 2, VAR_POLAR_SIGMOID = 3, VAR_SERIES_LIN = 4,
               VAR_ALL = 5 };
// op-tree layouts compiled into the column kernel: one union over 1 or 2
// extrusion classes; the difference of two unions over (1, 1) or (1, 2)
// classes; any other tree through the general composition program (4 or 8
// classes, at most kMaxNodes nodes).
enum Tree { TR_U1 = 0, TR_U2 = 1, TR_D11 = 2, TR_D12 = 3, TR_GEN4 = 4, TR_GEN8 = 5 };
__host__ __device__ constexpr int tree_nc(int tr) {
    return tr == TR_U1 ? 1 : tr == TR_U2 ? 2 : tr == TR_D11 ? 2 : tr == TR_D12 ? 3 : tr == TR_GEN4 ? 4 : 8;
}
// One primitive as the column kernel sees it.  The kernel works in (u, v, w)
// sample coordinates: u = x (lanes, contiguous in memory), v = the other
// in-plane axis and w = the column axis each thread walks.  Everything a
// primitive does along w is folded into its extrusion class.
struct DevPrim {
    int32_t type;          // SG_PRIM_*
    int32_t cls;           // extrusion class
    int32_t f0;            // first field of the primitive (flat field array)
    int32_t nvert;         // POLY / GCART vertices, POLAR Fourier order
    int32_t c0;            // first constant
    int32_t ubnd, vbnd;    // BOX: bounded along u / v
    int32_t fu0, fu1;      // BOX: fields of the u bounds
    int32_t fv0, fv1;      // BOX: fields of the v bounds
    int32_t sk0, sm0;      // sigma kind / k mode of argument 0 (u bound, boundary, x-range)
    int32_t sk1, sm1;      // sigma kind / k mode of argument 1 (v bound, GCART y boundary)
    union {
        int32_t gs0;       // GCART: first entry of its segment table (component 0, u = 0)
        // POLAR: its coefficient group, the index of the first primitive whose
        // 2 N Fourier coefficient fields are the same references (a, b, idx
        // alike: the same values and parameters)
        int32_t cgrp;
    };                     // others: -1
    double k0, k1;         // k_r (LOCAL) or k (FIXED)
    double reach0, reach1; // support half-width of each argument (um), for the support boxes
    double ax, ay;         // ELLIPSE aspect
    double iax, iay;       // 1 / aspect
};

// Segment of a piecewise-linear boundary (GCART) that a u-sample center falls
// in, and its position t in [0, 1] along it.  The vertices' x are constants of
// the scene, so the table is built once, per (primitive, component, u).
struct GSeg {
    int32_t j;
    int32_t pad;
    double t;
};

// Per-call copy of a primitive as the in-plane and partials kernels read it
// (written by k_stage): the record, its support box (u_lo, u_hi, v_lo, v_hi),
// and for boxes, ellipses and polar shapes the resolved values of their
// leading fields (boxes: u0 u1 v0 v1; ellipses: x0 y0 r; Fourier radius:
// x0 y0 R0; Polar2D: x0 y0 R delta) with the parameter index (-1:
// constant) and scale of each.
struct PrimRec {
    DevPrim pr;
    double4 bb;
    double f[4];
    double fb[4];
    int32_t fidx[4];
    int32_t pad[2];
};

// An extrusion class: primitives that are children of one op-tree node, with
// the same sign there (a difference's subtrahend enters its sum negated), and
// share the same factor along the column axis (a Rect1D in w, or 1).
struct DevClass {
    int32_t node;
    int32_t bounded;
    int32_t flo, fhi;      // fields of the w bounds
    int32_t skind, smode;
    double k;
};

struct StageParams {
    int32_t nprim, nclass, ncomp, nw;
    int64_t n_params;
    const sg_field* fref;
    const DevPrim* prims;
    const DevClass* cls;
    const double* consts;
    const double* p;
    int64_t pert_idx;            // parameter perturbed by +delta[variant] (-1: none)
    double delta[2];
    double* fval[2];
    float4* bbox[2];             // (u_lo, u_hi, v_lo, v_hi) of the support, rounded outward
    PrimRec* prec[2];
    double* ztab[2];             // [comp][class][w][3] = Z, dZ/dlo, dZ/dhi
    uint32_t* code[2];           // [comp][w] step codes
    uint32_t* gcode[2];          // [comp][group] group codes
    const double* wc[kMaxComp];  // column-axis sample centers / widths per component
    const double* ww[kMaxComp];
    int32_t nfield;
    int32_t tables;              // write the extrusion tables and codes (0: the scene's are static)
    double* zero_ptr;            // zeroed by variant 0 (gradient accumulator)
    int64_t zero_n;
    // F cache: variant 0's fields are compared with fprev (the fields the F
    // planes were computed from); any difference, or force, sets
    // chg[gen % 3]; chg[(gen + 1) % 3] is cleared for the next call.
    // fprev == nullptr: no comparison.
    const double* fprev;
    int32_t* chg;
    int32_t gen, force;
};

struct KParams {
    int32_t nu, nv, nw, ncomp;
    int64_t sv, sw, plane;       // element strides of v and w, elements per component plane
    int32_t tu, tv, tiles_u, tiles_v;        // in-plane tiles of the column kernel's blocks
    // 1: a block's samples are 256 consecutive in-plane samples (row-major,
    // rows joined: tiles_u = ceil(nu nv / 256), tiles_v = 1), so each
    // wavefront's samples are 64 consecutive elements of memory; eps_build
    // uses it when the rows are contiguous (sv == nu)
    int32_t linear;
    int32_t nseg, seglen;                    // column segments (seglen a multiple of kGroup)
    int32_t nprim, nclass;
    int32_t cls_wparam[kMaxClasses];
    // general composition program (TR_GEN*): nodes in postfix order, the root
    // last.  Node k sums sign_c F_c Z_c over its classes and sign_j v_j over
    // its child nodes, and applies its op: union min{1, S}, intersection
    // max{N - 1, S} - (N - 1), difference max{0, S}; a levels root chains its
    // child nodes in level order (Alg. cap).
    int32_t nnode, nlev;
    int32_t node_op[kMaxNodes];
    int32_t node_parent[kMaxNodes];        // -1 for the root
    int32_t cls_node[kMaxClasses];
    int32_t lev_node[kMaxNodes];           // levels root: the child node of each level
    double node_sign[kMaxNodes];           // +1, or -1 for a difference's subtrahend
    double node_nm1[kMaxNodes];            // intersection: number of children - 1
    double cls_sign[kMaxClasses];
    double lev_q[kMaxNodes];               // levels root: eps^{g-1} / eps^g (g >= 1)
    double eps_bg, deps;
    const double* uc[kMaxComp];
    const double* uw[kMaxComp];
    const double* vc[kMaxComp];
    const double* vw[kMaxComp];
    const DevPrim* prims;
    const DevClass* cls;
    const sg_field* fref;
    const double* consts;
    const GSeg* gseg;            // GCART segment tables
    const double* fval;
    const float4* bbox;
    const PrimRec* prec;
    const double* ztab;
    const double* fval2;         // FD: the second evaluation point
    const float4* bbox2;
    const PrimRec* prec2;
    const double* ztab2;
    const uint32_t* code;        // step codes [comp][w]
    const uint32_t* code2;
    const uint32_t* gcode;       // group codes [comp][group]
    const int32_t* grun;         // [comp][group]: the first group after it with another code (nullptr: none)
    const uint32_t* gcode2;
    float* out;                  // eps (MODE_EPS) or difference plane (MODE_FD)
    const float2* ef[kMaxComp];
    const float2* ea[kMaxComp];
    float two_omega;
    int32_t block0;              // k_column_batch: the request's first block in this launch (a slice of its blocks)
    const float* geps;
    double* grad;
    unsigned long long* nread;   // MODE_VJP_SPARSE: (sample, step) pairs whose fields were read, kReadSlots partial counts
    // MODE_FD_SPARSE: the perturbed parameter, its primitives (kprim[kprim_off[k] ..
    // kprim_off[k + 1]]), whether an extrusion bound references it (every tile
    // then takes part), and the difference scale 1 / (2h) or 1 / h
    int32_t fd_k, fd_all;
    const int32_t* kprim_off;
    const int32_t* kprim;
    double fd_scale;
    // deterministic reduction: each parameter sum goes into fx[3k .. 3k + 2]
    // as an exact fixed-point number (see fx_add); fx[3 n] flags a value out
    // of its range.  nullptr: FP64 atomics into grad.
    unsigned long long* fx;
    int64_t fx_n;
    // spread accumulation: block b adds into grad + (b mod kGradSpread) * gstride
    // (gstride = n: kGradSpread copies, summed by k_spread_finish; 0: one copy)
    int64_t gstride;
    // F cache (eps_build, eps_grad_vjp, eps_grad_vjp_geps): the in-plane sums
    // F_c of every sample as FP64 planes fplane[comp][class][v][u], valid
    // while chg[gen % 3] == 0 (no field differs from fprev, the nfield fields
    // they were computed from); a kernel that evaluates F writes both.
    // nullptr: no cache.
    double* fplane;
    double* fprev;
    const int32_t* chg;
    int32_t gen, nfield;
    // with the planes, each rectangular tile's candidate list: tlist[0] = the
    // tile width the lists are for (0 or -1: none), then per tile (block mod tiles) a
    // count (-1: more than one staging round) and kStageRec primitive indices
    int32_t* tlist;
};

// kernel launchers (sg_kernels.hip)
hipError_t launch_stage(const StageParams& sp, int nvariant, hipStream_t st);
// e0 / e1: optional events that take the kernel's own start and end times
hipError_t launch_column(int mode, int tree, int variant, const KParams& kp, hipStream_t st, hipEvent_t e0 = nullptr,
                         hipEvent_t e1 = nullptr);
// fused VJP (E, Eadj fields) over several requests of one kernel specialization:
// plist / first in device memory, blocks = first[nreq]
hipError_t launch_column_batch(int tree, int variant, const KParams* plist, const int* first, int nreq,
                               int64_t blocks, hipStream_t st);
// Philox4x32-10 N(0,1) complex64 planes (see shapegrad.h: sg_fieldgen), elements [i0, i1)
hipError_t launch_fieldgen(float2* e, float2* a, int64_t i0, int64_t i1, uint64_t seed, hipStream_t st);
hipError_t launch_gplane(const float2* const* ef, const float2* const* ea, int ncomp, int64_t plane,
                         float two_omega, float* g, hipStream_t st);
hipError_t launch_dot(const float* a, const float* b, int64_t n, double scale, double* out, hipStream_t st);
hipError_t launch_copy(void* dst, const void* src, int64_t bytes, hipStream_t st);
hipError_t launch_fill(double* dst, double v, int64_t n, hipStream_t st);
hipError_t launch_fx_finish(const unsigned long long* fx, int64_t n, double* grad, hipStream_t st);
hipError_t launch_spread_finish(const double* spread, int64_t n, double* grad, hipStream_t st);

}  // namespace sg

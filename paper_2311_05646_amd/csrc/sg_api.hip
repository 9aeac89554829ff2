// Host runtime of the C ABI declared in include/shapegrad.h: error state,
// contexts, the scene compiler (description -> device tables), staging of p
// and the entry points that enqueue the kernels of sg_kernels.hip.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "sg_device.h"
#include "sg_internal.h"
#include "sg_scene.h"

using namespace sg;

// ------------------------------------------------------------------ errors
static thread_local std::string g_err;

sg_status sg::fail(sg_status code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

extern "C" const char* sg_last_error(void) { return g_err.c_str(); }

// ------------------------------------------------------------------ scratch
// Per-call staging of eps_grad_vjp_noalloc (resolved fields, support boxes,
// primitive records, extrusion tables and step codes when they depend on p,
// spread gradient copies or fixed-point accumulators), for callers that
// cannot allocate device memory.  Each device holds its own copy for the life
// of the process; host code never uses this name as an address: sg_ctx_create
// takes the device address with hipGetSymbolAddress (sg_ctx::scratch).
constexpr int64_t kScratchBytes = int64_t(4) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// ------------------------------------------------------------------ context
extern "C" sg_status sg_ctx_create(int hip_device, sg_ctx** out) {
    if (!out) return fail(SG_E_INVALID, "sg_ctx_create: out is NULL");
    int n = 0;
    HIP_OK(hipGetDeviceCount(&n));
    if (hip_device < 0 || hip_device >= n) return fail(SG_E_INVALID, "sg_ctx_create: device %d of %d", hip_device, n);
    // the device address of this device's scratch array, taken with the
    // device current (every device holds its own copy)
    int prev = 0;
    HIP_OK(hipGetDevice(&prev));
    HIP_OK(hipSetDevice(hip_device));
    void* sp = nullptr;
    const hipError_t e = hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch));
    HIP_OK(hipSetDevice(prev));
    if (e != hipSuccess || !sp)
        return fail(SG_E_DEVICE, "sg_ctx_create: scratch address on device %d: %s", hip_device, hipGetErrorString(e));
    auto* c = new (std::nothrow) sg_ctx;
    if (!c) return fail(SG_E_NOMEM, "sg_ctx_create: out of host memory");
    c->device = hip_device;
    c->scratch = sp;
    *out = c;
    return SG_OK;
}

extern "C" void sg_ctx_destroy(sg_ctx* ctx) { delete ctx; }

static void axis_samples(const double* A, int64_t N, bool cell, std::vector<double>& c, std::vector<double>& w) {
    c.resize(N);
    w.resize(N);
    for (int64_t i = 0; i < N; ++i) {
        const double wi = A[i + 1] - A[i];
        if (cell) {
            c[i] = 0.5 * (A[i] + A[i + 1]);
            w[i] = wi;
        } else {
            const double wl = (i == 0) ? wi : (A[i] - A[i - 1]);
            c[i] = A[i];
            w[i] = 0.5 * (wl + wi);
        }
    }
}

static void free_scene(sg_scene* s) {
    if (!s) return;
    hipFree(s->d_lat);
    hipFree(s->d_fref);
    hipFree(s->d_prims);
    hipFree(s->d_cls);
    hipFree(s->d_consts);
    hipFree(s->d_gseg);
    hipFree(s->d_p);
    for (int i = 0; i < 2; ++i) {
        hipFree(s->d_fval[i]);
        hipFree(s->d_bbox[i]);
        hipFree(s->d_prec[i]);
        hipFree(s->d_ztab[i]);
        hipFree(s->d_code[i]);
        hipFree(s->d_gcode[i]);
        hipFree(s->d_work[i]);
    }
    hipFree(s->d_grad);
    hipFree(s->d_nread);
    hipFree(s->d_fx);
    hipFree(s->d_gspread);
    hipFree(s->d_fplane);
    hipFree(s->d_fprev);
    hipFree(s->d_grun);
    hipFree(s->d_tlist);
    hipFree(s->d_chg);
    hipFree(s->d_kprim_off);
    hipFree(s->d_kprim);
    if (s->h_p) hipHostFree(s->h_p);
    if (s->h_grad) hipHostFree(s->h_grad);
    if (s->p_evt) hipEventDestroy(s->p_evt);
    for (auto& r : s->recs) {
        hipEventDestroy(r.a);
        hipEventDestroy(r.b);
    }
    for (auto e : s->evpool) hipEventDestroy(e);
    delete s;
}

extern "C" void sg_scene_destroy(sg_scene* s) {
    if (!s) return;
    hipSetDevice(s->ctx->device);
    hipDeviceSynchronize();
    free_scene(s);
}

static bool valid_sigma(const sg_sigma& s) {
    return s.kind >= SG_SIGMA_SIGMOID && s.kind <= SG_SIGMA_QUADRATIC && (s.kmode == SG_K_LOCAL || s.kmode == SG_K_FIXED) &&
           std::isfinite(s.k) && s.k > 0.0;
}

static int expected_nfield(const sg_prim_desc& p) {
    switch (p.type) {
        case SG_PRIM_BOX: return 6;
        case SG_PRIM_ELLIPSE: return 5;
        case SG_PRIM_POLY: return 2 * p.nvert + 2;
        case SG_PRIM_GCART: return 2 * p.nvert + 4;
        case SG_PRIM_POLAR: return 2 * p.nvert + 5;
        case SG_PRIM_SERIES: return p.nvert + 4;
        case SG_PRIM_POLAR2D: return 6;
        default: return -1;
    }
}

// Field index (relative to the primitive) of the z extrusion bounds.
static int zfield(const sg_prim_desc& p) {
    switch (p.type) {
        case SG_PRIM_BOX: return 4;
        case SG_PRIM_ELLIPSE: return 3;
        case SG_PRIM_POLY: return 2 * p.nvert;
        case SG_PRIM_POLAR: return 2 * p.nvert + 3;
        case SG_PRIM_SERIES: return p.nvert + 2;
        case SG_PRIM_POLAR2D: return 4;
        default: return 2 * p.nvert + 2;
    }
}

struct ColSpec {
    int bounded;
    sg_field lo, hi;
    int kind, kmode;
    double k;
    bool operator==(const ColSpec& o) const {
        if (bounded != o.bounded) return false;
        if (!bounded) return true;
        return lo.a == o.lo.a && lo.b == o.lo.b && lo.idx == o.lo.idx && hi.a == o.hi.a && hi.b == o.hi.b &&
               hi.idx == o.hi.idx && kind == o.kind && kmode == o.kmode && k == o.k;
    }
};

extern "C" sg_status sg_scene_create(sg_ctx* ctx, const sg_scene_desc* d, sg_scene** out) {
    if (!ctx || !d || !out) return fail(SG_E_INVALID, "sg_scene_create: NULL argument");
    *out = nullptr;
    if (d->dim != 2 && d->dim != 3) return fail(SG_E_INVALID, "dim must be 2 or 3");
    if (d->ncomp < 1 || d->ncomp > 3) return fail(SG_E_INVALID, "ncomp must be 1..3");
    for (int c = 0; c < d->ncomp; ++c)
        if (d->comp_axis[c] < 0 || d->comp_axis[c] > 2) return fail(SG_E_INVALID, "comp_axis out of range");
    for (int a = 0; a < 3; ++a) {
        if (d->n[a] < 1 || d->n[a] > (1 << 24)) return fail(SG_E_INVALID, "n[%d] out of range", a);
        if (!d->nodes[a]) return fail(SG_E_INVALID, "nodes[%d] is NULL", a);
        for (int64_t i = 0; i < d->n[a]; ++i)
            if (!(d->nodes[a][i + 1] > d->nodes[a][i])) return fail(SG_E_INVALID, "nodes[%d] not increasing", a);
    }
    if (d->dim == 2 && d->n[2] != 1) return fail(SG_E_INVALID, "2D scenes have n[2] = 1");
    const int64_t plane = d->n[0] * d->n[1] * d->n[2];
    if (plane > ((int64_t)1 << 31)) return fail(SG_E_TOO_LARGE, "grid too large");
    if (d->n_params < 0) return fail(SG_E_INVALID, "n_params < 0");
    if (d->nprim < 1 || !d->prims) return fail(SG_E_INVALID, "no primitives");
    if (d->nfield < 0 || (d->nfield > 0 && !d->fields)) return fail(SG_E_INVALID, "fields");
    if (d->nconst < 0 || (d->nconst > 0 && !d->consts)) return fail(SG_E_INVALID, "consts");
    if (d->nnode < 1 || !d->nodes_op) return fail(SG_E_INVALID, "no op nodes");
    if (d->nchild < 1 || !d->children) return fail(SG_E_INVALID, "no children");
    for (int f = 0; f < d->nfield; ++f) {
        const sg_field& r = d->fields[f];
        if (r.idx >= d->n_params) return fail(SG_E_INVALID, "field %d references p[%lld] of %lld", f, (long long)r.idx,
                                              (long long)d->n_params);
        if (!std::isfinite(r.a) || !std::isfinite(r.b)) return fail(SG_E_INVALID, "field %d not finite", f);
    }
    // primitives
    for (int i = 0; i < d->nprim; ++i) {
        const sg_prim_desc& p = d->prims[i];
        const int nf = expected_nfield(p);
        if (nf < 0) return fail(SG_E_INVALID, "primitive %d: unknown type %d", i, p.type);
        if (p.type == SG_PRIM_POLY && (p.nvert < 3 || p.nvert > 64)) return fail(SG_E_INVALID, "poly %d: nvert", i);
        if (p.type == SG_PRIM_GCART && (p.nvert < 2 || p.nvert > 100000)) return fail(SG_E_INVALID, "gcart %d: nvert", i);
        if (p.type == SG_PRIM_POLAR && (p.nvert < 1 || p.nvert > 29)) return fail(SG_E_INVALID, "polar %d: order", i);
        if (p.type == SG_PRIM_SERIES && (p.nvert < 1 || p.nvert > 4096)) return fail(SG_E_INVALID, "series %d: terms", i);
        if (p.type == SG_PRIM_POLAR2D && (p.nvert < 1 || p.nvert > 64)) return fail(SG_E_INVALID, "polar2d %d: alpha", i);
        if (p.nfield != nf) return fail(SG_E_INVALID, "primitive %d: nfield %d, expected %d", i, p.nfield, nf);
        if (p.field_off < 0 || p.field_off + nf > d->nfield) return fail(SG_E_INVALID, "primitive %d: fields", i);
        const int nc = p.type == SG_PRIM_ELLIPSE ? 2 : p.type == SG_PRIM_GCART ? p.nvert : p.type == SG_PRIM_SERIES ? 5 : 0;
        if (p.nconst != nc || p.const_off < 0 || p.const_off + nc > d->nconst)
            return fail(SG_E_INVALID, "primitive %d: consts", i);
        const int nsig = p.type == SG_PRIM_BOX || p.type == SG_PRIM_GCART || p.type == SG_PRIM_SERIES ? 3 : 1;
        for (int a = 0; a < 3; ++a) {
            const bool used = (a < nsig) || (a == 2);
            const bool bnd = p.type == SG_PRIM_BOX ? p.bounded[a] != 0 : (a < 2 || p.bounded[2] != 0);
            if (used && bnd && !valid_sigma(p.sigma[a])) return fail(SG_E_INVALID, "primitive %d: sigma[%d]", i, a);
        }
        if (d->dim == 2 && p.bounded[2]) return fail(SG_E_INVALID, "primitive %d: bounded along z in a 2D scene", i);
        if ((p.type == SG_PRIM_ELLIPSE || p.type == SG_PRIM_POLY || p.type == SG_PRIM_POLAR ||
             p.type == SG_PRIM_POLAR2D) &&
            p.sigma[0].kmode != SG_K_FIXED)
            return fail(SG_E_INVALID, "primitive %d: radial/oblique boundary needs a FIXED k", i);
        if (p.type == SG_PRIM_ELLIPSE) {
            const double ax = d->consts[p.const_off], ay = d->consts[p.const_off + 1];
            if (!(ax > 0) || !(ay > 0)) return fail(SG_E_INVALID, "ellipse %d: aspect must be > 0", i);
        }
        if (p.type == SG_PRIM_SERIES && !(d->consts[p.const_off + 1] > 0.0))
            return fail(SG_E_INVALID, "series %d: L must be > 0", i);
        if (p.type == SG_PRIM_GCART)
            for (int j = 0; j + 1 < p.nvert; ++j)
                if (!(d->consts[p.const_off + j + 1] > d->consts[p.const_off + j]))
                    return fail(SG_E_INVALID, "gcart %d: vertex x not increasing", i);
    }
    // op tree -> nodes (postfix, root last), each with the primitives among
    // its children (and the sign they enter its sum with) and its child nodes
    struct HNode {
        int op = SG_OP_UNION;
        int parent = -1;
        double sign = 1.0;
        int nchild = 0;
        std::vector<int> prims;
        std::vector<double> psign;
    };
    auto child = [&](const sg_node_desc& nd, int c) -> int { return d->children[nd.child_off + c]; };
    for (int k = 0; k < d->nnode; ++k) {
        const sg_node_desc& nd = d->nodes_op[k];
        if (nd.op < SG_OP_UNION || nd.op > SG_OP_LEVELS) return fail(SG_E_INVALID, "node %d: op", k);
        if (nd.op == SG_OP_LEVELS && k != d->nnode - 1) return fail(SG_E_INVALID, "node %d: levels must be the root", k);
        if (nd.nchild < 1 || nd.child_off < 0 || nd.child_off + nd.nchild > d->nchild)
            return fail(SG_E_INVALID, "node %d: children", k);
        if (nd.op == SG_OP_DIFFERENCE && nd.nchild != 2) return fail(SG_E_INVALID, "node %d: difference takes 2", k);
        for (int c = 0; c < nd.nchild; ++c) {
            const int ch = child(nd, c);
            if (ch >= d->nprim) return fail(SG_E_INVALID, "node %d: primitive %d out of range", k, ch);
            if (ch < 0 && -(ch + 1) >= k) return fail(SG_E_INVALID, "node %d: child node must come earlier", k);
        }
    }
    std::vector<HNode> hn;
    std::vector<int> map(d->nnode, -1);       // description node -> hn index
    std::vector<int> used(d->nprim, 0);
    const sg_node_desc& root = d->nodes_op[d->nnode - 1];
    const bool levels = root.op == SG_OP_LEVELS;
    double lev_q[kMaxNodes] = {};
    std::vector<int> lev_child;               // hn index of each level's node
    for (int k = 0; k < d->nnode; ++k) {
        const sg_node_desc& nd = d->nodes_op[k];
        const bool is_root = k == d->nnode - 1;
        if (is_root && levels) {
            const int K = nd.nchild;
            if (K < 2 || K > kMaxNodes - 1) return fail(SG_E_UNSUPPORTED, "levels: 2 to %d material sets", kMaxNodes - 1);
            if (nd.aux < 0 || nd.aux + K > d->nconst) return fail(SG_E_INVALID, "levels: level values out of consts");
            const double* lv = d->consts + nd.aux;
            for (int c = 0; c < K; ++c) {
                if (!(lv[c] > 0.0) || !std::isfinite(lv[c]) || (c > 0 && lv[c] < lv[c - 1]))
                    return fail(SG_E_INVALID, "levels: values must be positive and ascending");
                lev_q[c] = c == 0 ? 1.0 : lv[c - 1] / lv[c];
            }
            const double top = d->eps_fg - d->eps_bg;
            if (std::fabs(lv[K - 1] - top) > 1e-12 * std::max(1.0, std::fabs(top)))
                return fail(SG_E_INVALID, "levels: the top level must equal eps_fg - eps_bg");
            // every material set becomes a node: a primitive child is a union of one
            for (int c = 0; c < K; ++c) {
                const int ch = child(nd, c);
                if (ch >= 0) {
                    HNode w;
                    w.nchild = 1;
                    w.prims.push_back(ch);
                    w.psign.push_back(1.0);
                    hn.push_back(w);
                    lev_child.push_back((int)hn.size() - 1);
                } else {
                    const int j = map[-(ch + 1)];
                    if (hn[j].parent >= 0) return fail(SG_E_INVALID, "node %d has two parents", -(ch + 1));
                    if (hn[j].op == SG_OP_LEVELS) return fail(SG_E_INVALID, "levels must be the root");
                    lev_child.push_back(j);
                }
            }
            HNode r;
            r.op = SG_OP_LEVELS;
            r.nchild = K;
            hn.push_back(r);
            for (int j : lev_child) hn[j].parent = (int)hn.size() - 1;
            map[k] = (int)hn.size() - 1;
            continue;
        }
        HNode h;
        h.op = nd.op;
        h.nchild = nd.nchild;
        const int me = (int)hn.size();
        for (int c = 0; c < nd.nchild; ++c) {
            const int ch = child(nd, c);
            const double sg = (nd.op == SG_OP_DIFFERENCE && c == 1) ? -1.0 : 1.0;
            if (ch >= 0) {
                h.prims.push_back(ch);
                h.psign.push_back(sg);
            } else {
                const int j = map[-(ch + 1)];
                if (hn[j].parent >= 0) return fail(SG_E_INVALID, "node %d has two parents", -(ch + 1));
                hn[j].parent = me;
                hn[j].sign = sg;
            }
        }
        hn.push_back(h);
        map[k] = me;
    }
    // every node must hang below the root
    for (int j = 0; j + 1 < (int)hn.size(); ++j)
        if (hn[j].parent < 0) return fail(SG_E_INVALID, "op node %d is not below the root", j);
    if ((int)hn.size() > kMaxNodes)
        return fail(SG_E_UNSUPPORTED, "the op tree has %d nodes (the GPU composition takes at most %d)", (int)hn.size(),
                    kMaxNodes);
    for (auto& h : hn)
        for (int pi : h.prims) {
            if (used[pi]) return fail(SG_E_INVALID, "primitive %d appears twice in the tree", pi);
            used[pi] = 1;
        }
    // the order classes are numbered in: a depth-first walk from the root,
    // children in order, so a difference's minuend side comes first
    std::vector<std::pair<int, int>> class_order;     // (hn node, index into its prims)
    {
        std::vector<std::vector<int>> kids(hn.size());
        for (int j = 0; j + 1 < (int)hn.size(); ++j) kids[hn[j].parent].push_back(j);
        // children of a description node in their given order: primitives
        // and child nodes interleave as listed
        std::vector<std::vector<std::pair<int, int>>> items(hn.size());   // (0 prim idx | 1 node, value)
        for (int k = 0; k < d->nnode; ++k) {
            const int me = map[k];
            const sg_node_desc& nd = d->nodes_op[k];
            if (hn[me].op == SG_OP_LEVELS) {
                for (int j : lev_child) items[me].push_back({1, j});
                continue;
            }
            int pc = 0;
            for (int c = 0; c < nd.nchild; ++c) {
                const int ch = child(nd, c);
                if (ch >= 0) items[me].push_back({0, pc++});
                else items[me].push_back({1, map[-(ch + 1)]});
            }
        }
        for (int j : lev_child)
            if (items[j].empty() && hn[j].prims.size() == 1) items[j].push_back({0, 0});
        std::function<void(int)> walk = [&](int k) {
            for (auto& it : items[k]) {
                if (it.first == 0) class_order.push_back({k, it.second});
                else walk(it.second);
            }
        };
        walk((int)hn.size() - 1);
    }

    // column axis: y for 2D scenes made only of boxes whose y-extents form at
    // most kMaxClasses classes (the boxes' y factor then becomes the column
    // factor), else z
    bool all_box = true;
    for (int i = 0; i < d->nprim; ++i)
        if (used[i] && d->prims[i].type != SG_PRIM_BOX) all_box = false;
    bool y_classes_fit = true;
    if (d->dim == 2 && all_box) {
        // classes are (node, sign, y factor) when y is the column axis
        std::vector<std::tuple<int, double, ColSpec>> seen;
        for (auto& [k, i] : class_order) {
            const sg_prim_desc& p = d->prims[hn[k].prims[i]];
            ColSpec cs{};
            cs.bounded = p.bounded[1] != 0;
            if (cs.bounded) {
                cs.lo = d->fields[p.field_off + 2];
                cs.hi = d->fields[p.field_off + 3];
                cs.kind = p.sigma[1].kind;
                cs.kmode = p.sigma[1].kmode;
                cs.k = p.sigma[1].k;
            }
            bool found = false;
            for (auto& t : seen)
                if (std::get<0>(t) == k && std::get<1>(t) == hn[k].psign[i] && std::get<2>(t) == cs) found = true;
            if (!found) seen.emplace_back(k, hn[k].psign[i], cs);
        }
        y_classes_fit = (int)seen.size() <= kMaxClasses;
    }
    const int col = (d->dim == 2 && all_box && y_classes_fit) ? 1 : 2;
    const int axis_v = col == 2 ? 1 : 2;

    auto* s = new (std::nothrow) sg_scene;
    if (!s) return fail(SG_E_NOMEM, "host memory");
    s->ctx = ctx;
    s->dim = d->dim;
    s->ncomp = d->ncomp;
    for (int c = 0; c < 3; ++c) s->comp_axis[c] = d->comp_axis[c];
    for (int a = 0; a < 3; ++a) s->n[a] = d->n[a];
    s->n_params = d->n_params;
    s->nfield = d->nfield;
    s->eps_bg = d->eps_bg;
    s->eps_fg = d->eps_fg;
    s->col = col;
    s->axis_v = axis_v;
    s->nu = (int)d->n[0];
    s->nv = (int)d->n[axis_v];
    s->nw = (int)d->n[col];
    const int64_t stride[3] = {1, d->n[0], d->n[0] * d->n[1]};
    s->sv = stride[axis_v];
    s->sw = stride[col];
    s->plane = plane;
    // the stream kernel addresses 8 column steps of complex64 samples from one
    // buffer resource with 32-bit offsets
    if (s->sw * 8 * 8 >= ((int64_t)1 << 31)) {
        free_scene(s);
        return fail(SG_E_TOO_LARGE, "the plane across the column axis holds %lld samples (limit %lld)",
                    (long long)s->sw, (long long)(((int64_t)1 << 31) / 64 - 1));
    }
    s->fields.assign(d->fields, d->fields + d->nfield);

    // extrusion classes
    auto colspec = [&](int pi) {
        const sg_prim_desc& p = d->prims[pi];
        ColSpec cs{};
        int fz, sa;
        if (p.type == SG_PRIM_BOX) {
            fz = 2 * col;
            sa = col;
            cs.bounded = p.bounded[col] != 0;
        } else {
            fz = zfield(p);
            sa = 2;
            cs.bounded = p.bounded[2] != 0;
        }
        if (cs.bounded) {
            cs.lo = d->fields[p.field_off + fz];
            cs.hi = d->fields[p.field_off + fz + 1];
            cs.kind = p.sigma[sa].kind;
            cs.kmode = p.sigma[sa].kmode;
            cs.k = p.sigma[sa].k;
        }
        return std::make_tuple(cs, p.field_off + fz);
    };
    std::vector<int> prim_cls(d->nprim, -1);
    std::vector<ColSpec> specs;
    for (auto& [k, i] : class_order) {
        const int pi = hn[k].prims[i];
        const double sg = hn[k].psign[i];
        auto [cs, fz] = colspec(pi);
        int found = -1;
        for (int c = 0; c < (int)specs.size(); ++c)
            if (s->classes[c].node == k && s->cls_sign[c] == sg && specs[c] == cs) found = c;
        if (found < 0) {
            if ((int)specs.size() == kMaxClasses) {
                free_scene(s);
                return fail(SG_E_UNSUPPORTED, "more than %d extrusion classes", kMaxClasses);
            }
            found = (int)specs.size();
            specs.push_back(cs);
            DevClass dc{};
            dc.node = k;
            dc.bounded = cs.bounded;
            dc.flo = cs.bounded ? fz : -1;
            dc.fhi = cs.bounded ? fz + 1 : -1;
            dc.skind = cs.kind;
            dc.smode = cs.kmode;
            dc.k = cs.bounded ? cs.k : 1.0;
            s->classes.push_back(dc);
            s->cls_sign.push_back(sg);
        }
        prim_cls[pi] = found;
    }
    s->nclass = (int)s->classes.size();
    s->ncls_pad = s->nclass <= 1 ? 1 : s->nclass <= 2 ? 2 : s->nclass <= 4 ? 4 : 8;
    s->nnode = (int)hn.size();
    for (int k = 0; k < s->nnode; ++k) {
        s->node_op[k] = hn[k].op;
        s->node_parent[k] = hn[k].parent;
        s->node_sign[k] = hn[k].sign;
        s->node_nm1[k] = (double)(hn[k].nchild - 1);
    }
    s->nlev = (int)lev_child.size();
    for (int g = 0; g < s->nlev; ++g) {
        s->lev_node[g] = lev_child[g];
        s->lev_q[g] = lev_q[g];
    }

    // lattices and the largest sample width per in-plane axis
    std::vector<double> lat;
    double wmax[3] = {0, 0, 0};
    for (int c = 0; c < d->ncomp; ++c) {
        const int axes[3] = {0, axis_v, col};
        for (int q = 0; q < 3; ++q) {
            const int a = axes[q];
            std::vector<double> cc, ww;
            axis_samples(d->nodes[a], d->n[a], a == d->comp_axis[c], cc, ww);
            for (double w : ww) wmax[a] = std::max(wmax[a], w);
            s->lat_off[c][2 * q] = (int64_t)lat.size();
            lat.insert(lat.end(), cc.begin(), cc.end());
            s->lat_off[c][2 * q + 1] = (int64_t)lat.size();
            lat.insert(lat.end(), ww.begin(), ww.end());
        }
    }
    // device primitive records (primitives of the tree only, in index order)
    std::vector<DevPrim> prims;
    std::vector<GSeg> gseg;     // piecewise-linear boundaries: segment of every u-sample center
    std::map<std::string, int32_t> cgroups;     // Fourier coefficient fields (bytes) -> first primitive
    for (int i = 0; i < d->nprim; ++i) {
        if (!used[i]) continue;
        const sg_prim_desc& p = d->prims[i];
        DevPrim r{};
        r.type = p.type;
        r.cls = prim_cls[i];
        r.f0 = p.field_off;
        r.nvert = p.nvert;
        r.c0 = p.const_off;
        auto reach = [&](const sg_sigma& sgm, int axis) {
            const double k = sgm.kmode == SG_K_LOCAL ? sgm.k / wmax[axis] : sgm.k;
            return sigma_cut(sgm.kind) / k;
        };
        r.gs0 = -1;
        if (p.type == SG_PRIM_POLAR) {
            std::string key(reinterpret_cast<const char*>(&p.nvert), sizeof(p.nvert));
            key.append(reinterpret_cast<const char*>(d->fields + p.field_off + 3), 2 * p.nvert * sizeof(sg_field));
            auto it = cgroups.find(key);
            r.cgrp = it != cgroups.end() ? it->second : (int32_t)prims.size();
            if (it == cgroups.end()) cgroups.emplace(std::move(key), r.cgrp);
        }
        if (p.type == SG_PRIM_GCART) {
            // largest j in [0, M-2] with x_j <= x (0 left of the first vertex),
            // and t = (x - x_j) / (x_{j+1} - x_j) clamped to [0, 1]
            const double* xv = d->consts + p.const_off;
            const int M = p.nvert;
            r.gs0 = (int32_t)gseg.size();
            for (int c = 0; c < d->ncomp; ++c) {
                const double* uc = lat.data() + s->lat_off[c][0];
                for (int u = 0; u < s->nu; ++u) {
                    int j = 0;
                    while (j + 1 <= M - 2 && xv[j + 1] <= uc[u]) ++j;
                    const double tt = (uc[u] - xv[j]) / (xv[j + 1] - xv[j]);
                    GSeg g{};
                    g.j = j;
                    g.t = std::min(1.0, std::max(0.0, tt));
                    gseg.push_back(g);
                }
            }
        }
        if (p.type == SG_PRIM_BOX) {
            r.ubnd = p.bounded[0] != 0;
            r.vbnd = p.bounded[axis_v] != 0;
            r.fu0 = p.field_off + 0;
            r.fu1 = p.field_off + 1;
            r.fv0 = p.field_off + 2 * axis_v;
            r.fv1 = p.field_off + 2 * axis_v + 1;
            r.sk0 = p.sigma[0].kind;
            r.sm0 = p.sigma[0].kmode;
            r.k0 = p.sigma[0].k;
            r.sk1 = p.sigma[axis_v].kind;
            r.sm1 = p.sigma[axis_v].kmode;
            r.k1 = p.sigma[axis_v].k;
            r.reach0 = r.ubnd ? reach(p.sigma[0], 0) : 0.0;
            r.reach1 = r.vbnd ? reach(p.sigma[axis_v], axis_v) : 0.0;
        } else {
            r.ubnd = r.vbnd = 1;
            r.sk0 = p.sigma[0].kind;
            r.sm0 = p.sigma[0].kmode;
            r.k0 = p.sigma[0].k;
            r.reach0 = reach(p.sigma[0], 0);
            if (p.type == SG_PRIM_GCART || p.type == SG_PRIM_SERIES) {
                r.sk1 = p.sigma[1].kind;
                r.sm1 = p.sigma[1].kmode;
                r.k1 = p.sigma[1].k;
                r.reach1 = reach(p.sigma[1], 1);
            }
            if (p.type == SG_PRIM_ELLIPSE) {
                r.ax = d->consts[p.const_off];
                r.ay = d->consts[p.const_off + 1];
                r.iax = 1.0 / r.ax;
                r.iay = 1.0 / r.ay;
            }
        }
        prims.push_back(r);
    }
    // parameter -> primitives (device order) and parameter -> extrusion bound
    {
        std::vector<std::vector<int32_t>> lists(std::max<int64_t>(1, d->n_params));
        int dev = 0;
        for (int i = 0; i < d->nprim; ++i) {
            if (!used[i]) continue;
            const sg_prim_desc& p = d->prims[i];
            for (int f = 0; f < p.nfield; ++f) {
                const int64_t k = d->fields[p.field_off + f].idx;
                if (k >= 0 && (lists[k].empty() || lists[k].back() != dev)) lists[k].push_back(dev);
            }
            ++dev;
        }
        s->kprim_off.assign(1, 0);
        for (const auto& l : lists) {
            s->kprim.insert(s->kprim.end(), l.begin(), l.end());
            s->kprim_off.push_back((int32_t)s->kprim.size());
        }
        s->k_wbound.assign(std::max<int64_t>(1, d->n_params), 0);
        for (const DevClass& c : s->classes) {
            if (!c.bounded) continue;
            for (int f : {c.flo, c.fhi})
                if (s->fields[f].idx >= 0) s->k_wbound[s->fields[f].idx] = 1;
        }
    }
    s->nprim = (int)prims.size();
    // smallest kernel variant covering the primitive types and in-plane sigma kinds
    {
        int tmask = 0, smask = 0;
        for (int i = 0; i < d->nprim; ++i) {
            if (!used[i]) continue;
            const sg_prim_desc& p = d->prims[i];
            tmask |= p.type == SG_PRIM_POLAR2D ? T_POLAR : 1 << p.type;     // one radial feature set
            if (p.type == SG_PRIM_BOX) {
                if (p.bounded[0]) smask |= sigma_bit(p.sigma[0].kind);
                if (p.bounded[axis_v]) smask |= sigma_bit(p.sigma[axis_v].kind);
            } else {
                smask |= sigma_bit(p.sigma[0].kind);
                if (p.type == SG_PRIM_GCART || p.type == SG_PRIM_SERIES) smask |= sigma_bit(p.sigma[1].kind);
            }
        }
        const int vt[5] = {T_BOX, T_BOX | T_GCART, T_BOX | T_ELL, T_BOX | T_POLAR, T_BOX | T_SERIES};
        const int vs[5] = {S_LIN, S_LIN, S_LIN | S_SIGMOID, S_LIN | S_SIGMOID, S_LIN};
        s->variant = VAR_ALL;
        for (int v = 0; v < 5; ++v)
            if ((tmask & ~vt[v]) == 0 && (smask & ~vs[v]) == 0) { s->variant = v; break; }
        // op-tree layout: the fixed ones need every node to be a plain union
        // (or a single-primitive node) over primitives only
        auto plain = [&](int k) {
            return (hn[k].op == SG_OP_UNION || hn[k].nchild == 1) && (int)hn[k].prims.size() == hn[k].nchild;
        };
        int ncls_node[kMaxNodes] = {};
        bool neg_cls = false;
        for (int c = 0; c < s->nclass; ++c) {
            ncls_node[s->classes[c].node]++;
            neg_cls = neg_cls || s->cls_sign[c] < 0.0;
        }
        const int rt = s->nnode - 1;
        s->tree = s->nclass <= 4 ? TR_GEN4 : TR_GEN8;
        if (s->nnode == 1 && plain(0) && !neg_cls) {
            if (s->nclass == 1) s->tree = TR_U1;
            else if (s->nclass == 2) s->tree = TR_U2;
        } else if (hn[rt].op == SG_OP_DIFFERENCE && s->nnode <= 3) {
            // difference of (a primitive or a plain union) and (a primitive or a
            // plain union); class 0 is the minuend's, the rest the subtrahend's
            bool ok = true;
            int nsub = 0;
            for (int k = 0; k < rt; ++k) ok = ok && plain(k) && hn[k].parent == rt;
            for (int c = 0; c < s->nclass && ok; ++c) {
                const int k = s->classes[c].node;
                const bool minuend = (k == rt) ? s->cls_sign[c] > 0.0 : hn[k].sign > 0.0;
                if (k != rt && s->cls_sign[c] < 0.0) ok = false;
                if ((c == 0) != minuend) ok = false;
                if (!minuend) ++nsub;
            }
            if (ok && nsub == 1) s->tree = TR_D11;
            else if (ok && nsub == 2) s->tree = TR_D12;
        }
        if (s->tree == TR_GEN4 || s->tree == TR_GEN8) s->variant = VAR_ALL;
    }

    // device allocations
    hipError_t e = hipSetDevice(ctx->device);
    auto alloc = [&](void** ptr, size_t bytes) {
        if (e == hipSuccess) e = hipMalloc(ptr, std::max<size_t>(bytes, 16));
    };
    alloc((void**)&s->d_lat, lat.size() * sizeof(double));
    alloc((void**)&s->d_fref, std::max<int64_t>(1, d->nfield) * sizeof(sg_field));
    alloc((void**)&s->d_prims, prims.size() * sizeof(DevPrim));
    alloc((void**)&s->d_kprim_off, s->kprim_off.size() * sizeof(int32_t));
    alloc((void**)&s->d_kprim, std::max<size_t>(1, s->kprim.size()) * sizeof(int32_t));
    alloc((void**)&s->d_cls, s->classes.size() * sizeof(DevClass));
    alloc((void**)&s->d_consts, std::max(1, d->nconst) * sizeof(double));
    alloc((void**)&s->d_gseg, std::max<size_t>(1, gseg.size()) * sizeof(GSeg));
    alloc((void**)&s->d_p, std::max<int64_t>(1, d->n_params) * sizeof(double));
    alloc((void**)&s->d_grad, std::max<int64_t>(1, d->n_params) * sizeof(double));
    for (int v = 0; v < 2; ++v) {
        alloc((void**)&s->d_fval[v], std::max<int64_t>(1, d->nfield) * sizeof(double));
        alloc((void**)&s->d_bbox[v], prims.size() * sizeof(float4));
        alloc((void**)&s->d_prec[v], prims.size() * sizeof(PrimRec));
        alloc((void**)&s->d_ztab[v], (size_t)d->ncomp * s->nclass * s->nw * 3 * sizeof(double));
        alloc((void**)&s->d_code[v], (size_t)d->ncomp * s->nw * sizeof(uint32_t));
        alloc((void**)&s->d_gcode[v], (size_t)d->ncomp * ((s->nw + kGroup - 1) / kGroup) * sizeof(uint32_t));
    }
    if (e == hipSuccess) e = hipHostMalloc((void**)&s->h_p, std::max<int64_t>(1, d->n_params) * sizeof(double));
    if (e == hipSuccess) e = hipHostMalloc((void**)&s->h_grad, std::max<int64_t>(1, d->n_params) * sizeof(double));
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->p_evt, hipEventDisableTiming);
    if (e == hipSuccess) e = hipMemcpy(s->d_lat, lat.data(), lat.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess && d->nfield)
        e = hipMemcpy(s->d_fref, d->fields, d->nfield * sizeof(sg_field), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(s->d_prims, prims.data(), prims.size() * sizeof(DevPrim), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(s->d_kprim_off, s->kprim_off.data(), s->kprim_off.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess && !s->kprim.empty())
        e = hipMemcpy(s->d_kprim, s->kprim.data(), s->kprim.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(s->d_cls, s->classes.data(), s->classes.size() * sizeof(DevClass), hipMemcpyHostToDevice);
    if (e == hipSuccess && d->nconst)
        e = hipMemcpy(s->d_consts, d->consts, d->nconst * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess && !gseg.empty())
        e = hipMemcpy(s->d_gseg, gseg.data(), gseg.size() * sizeof(GSeg), hipMemcpyHostToDevice);
    // shared parameters: one referenced by at least 8 primitives, or a term
    // of a sine-series boundary (which every block on the boundary reaches)
    for (int64_t k = 0; k < d->n_params && !s->spread; ++k)
        if (s->kprim_off[k + 1] - s->kprim_off[k] >= 8) s->spread = true;
    for (int i = 0; i < d->nprim && !s->spread; ++i)
        if (d->prims[i].type == SG_PRIM_SERIES) s->spread = true;
    if (s->spread) alloc((void**)&s->d_gspread, (size_t)kGradSpread * std::max<int64_t>(1, d->n_params) * sizeof(double));
    // static extrusion tables: one stage launch with no primitive, on the null
    // stream, finished before the scene is returned
    s->static_w = true;
    for (const DevClass& c : s->classes)
        if (c.bounded && (s->fields[c.flo].idx >= 0 || s->fields[c.fhi].idx >= 0)) s->static_w = false;
    if (e == hipSuccess && s->static_w) {
        StageParams sp = stage_params(s, s->d_p);
        sp.nprim = 0;
        sp.tables = 1;
        e = launch_stage(sp, 1, nullptr);
        if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
        // runs of equal group codes: grun[comp][g] = the first group after g
        // whose code differs (eps_build stores a run with no per-group code)
        const int ngw = (s->nw + kGroup - 1) / kGroup;
        std::vector<uint32_t> gc((size_t)s->ncomp * ngw);
        std::vector<int32_t> run(gc.size());
        if (e == hipSuccess) e = hipMemcpy(gc.data(), s->d_gcode[0], gc.size() * sizeof(uint32_t), hipMemcpyDeviceToHost);
        if (e == hipSuccess) {
            for (int c = 0; c < s->ncomp; ++c) {
                const uint32_t* g = gc.data() + (size_t)c * ngw;
                int32_t* r = run.data() + (size_t)c * ngw;
                for (int i = ngw - 1; i >= 0; --i) r[i] = (i + 1 < ngw && g[i + 1] == g[i]) ? r[i + 1] : i + 1;
            }
            e = hipMalloc((void**)&s->d_grun, run.size() * sizeof(int32_t));
            if (e == hipSuccess) e = hipMemcpy(s->d_grun, run.data(), run.size() * sizeof(int32_t), hipMemcpyHostToDevice);
        }
    }
    if (e != hipSuccess) {
        free_scene(s);
        return fail(e == hipErrorOutOfMemory ? SG_E_NOMEM : SG_E_DEVICE, "sg_scene_create: %s", hipGetErrorString(e));
    }
    {
        const char* det = std::getenv("SG_DETERMINISTIC");
        s->deterministic = det != nullptr && std::atoi(det) != 0;
        const char* rect = std::getenv("SG_EPS_RECT_TILES");
        s->linear_tiles = !(rect != nullptr && std::atoi(rect) != 0);
        // the F cache pays where the in-plane evaluation is costly (sigmoid
        // ellipses, Fourier radii, sine series, the catch-all set): measured
        // on the Fourier-scatterer coupler, gradient after eps_build 200 ->
        // 169 us; with boxes and piecewise-linear boundaries its plane traffic
        // costs about what it saves (taper: 183.5 vs 187.9 us per step)
        const char* fc = std::getenv("SG_F_CACHE");
        if (fc != nullptr) s->fcache = std::atoi(fc) != 0;
        else s->fcache = !(s->variant == VAR_BOX_LIN || s->variant == VAR_GCART_LIN);
    }
    *out = s;
    return SG_OK;
}

extern "C" sg_status sg_scene_info(const sg_scene* s, int64_t* n_params, int32_t* ncomp, int64_t dims[3]) {
    if (!s) return fail(SG_E_INVALID, "sg_scene_info: NULL scene");
    if (n_params) *n_params = s->n_params;
    if (ncomp) *ncomp = s->ncomp;
    if (dims)
        for (int a = 0; a < 3; ++a) dims[a] = s->n[a];
    return SG_OK;
}

extern "C" sg_status sg_scene_set_launch(sg_scene* s, int32_t block_x, int32_t col_segments) {
    if (!s) return fail(SG_E_INVALID, "NULL scene");
    if (block_x != 0 && block_x != 16 && block_x != 32 && block_x != 64 && block_x != 128 && block_x != 256)
        return fail(SG_E_INVALID, "block_x must be 0, 16, 32, 64, 128 or 256");
    if (col_segments < 0) return fail(SG_E_INVALID, "col_segments < 0");
    std::lock_guard<std::mutex> lk(s->mu);
    s->block_x = block_x;
    s->nseg = col_segments;
    return SG_OK;
}

// ------------------------------------------------------------------ calls
static sg_status stage_p(sg_scene* s, const double* p, int p_on_device, hipStream_t st, const double** dp) {
    if (s->n_params == 0) {
        *dp = s->d_p;
        return SG_OK;
    }
    if (!p) return fail(SG_E_INVALID, "p is NULL");
    if (p_on_device) {
        *dp = p;
        return SG_OK;
    }
    for (int64_t i = 0; i < s->n_params; ++i)
        if (!std::isfinite(p[i])) return fail(SG_E_INVALID, "p[%lld] is not finite", (long long)i);
    if (s->p_evt_pending) HIP_OK(hipEventSynchronize(s->p_evt));
    std::memcpy(s->h_p, p, s->n_params * sizeof(double));
    HIP_OK(hipMemcpyAsync(s->d_p, s->h_p, s->n_params * sizeof(double), hipMemcpyHostToDevice, st));
    HIP_OK(hipEventRecord(s->p_evt, st));
    s->p_evt_pending = true;
    *dp = s->d_p;
    return SG_OK;
}

StageParams sg::stage_params(sg_scene* s, const double* dp) {
    StageParams sp{};
    sp.nprim = s->nprim;
    sp.nclass = s->nclass;
    sp.ncomp = s->ncomp;
    sp.nw = s->nw;
    sp.n_params = s->n_params;
    sp.fref = s->d_fref;
    sp.prims = s->d_prims;
    sp.cls = s->d_cls;
    sp.consts = s->d_consts;
    sp.p = dp;
    sp.pert_idx = -1;
    sp.delta[0] = sp.delta[1] = 0.0;
    for (int v = 0; v < 2; ++v) {
        sp.fval[v] = s->d_fval[v];
        sp.bbox[v] = s->d_bbox[v];
        sp.prec[v] = s->d_prec[v];
        sp.ztab[v] = s->d_ztab[v];
        sp.code[v] = s->d_code[v];
        sp.gcode[v] = s->d_gcode[v];
    }
    for (int c = 0; c < kMaxComp; ++c) {
        const int cc = std::min(c, s->ncomp - 1);
        sp.wc[c] = s->d_lat + s->lat_off[cc][4];
        sp.ww[c] = s->d_lat + s->lat_off[cc][5];
    }
    sp.nfield = (int)s->nfield;
    sp.tables = s->static_w ? 0 : 1;
    sp.zero_ptr = nullptr;
    sp.zero_n = 0;
    return sp;
}

KParams sg::column_params(sg_scene* s, int64_t target_blocks, bool linear) {
    KParams kp{};
    kp.nu = s->nu;
    kp.nv = s->nv;
    kp.nw = s->nw;
    kp.ncomp = s->ncomp;
    kp.sv = s->sv;
    kp.sw = s->sw;
    kp.plane = s->plane;
    // square tiles when many primitives compete for a tile, wide rows of x
    // (contiguous field bytes per column step) otherwise
    int tu = s->block_x;
    if (tu == 0) tu = (s->nv == 1) ? 256 : (s->nprim > 32 ? 16 : 128);
    kp.tu = tu;
    kp.tv = kBlock / tu;
    kp.tiles_u = (s->nu + tu - 1) / tu;
    kp.tiles_v = (s->nv + kp.tv - 1) / kp.tv;
    // linear tiles only where the automatic choice is wide rows: with many
    // small primitives a 64-sample strip per wavefront meets about twice as
    // many of them as a 16 x 4 patch (measured: eps_build on the 1601-hole
    // grating 59 -> 108 us)
    if (linear && s->sv == s->nu && s->linear_tiles && s->block_x == 0 && tu >= 128) {
        kp.linear = 1;
        kp.tu = kBlock;
        kp.tv = 1;
        kp.tiles_u = (int32_t)(((int64_t)s->nu * s->nv + kBlock - 1) / kBlock);
        kp.tiles_v = 1;
    }
    int nseg = s->nseg;
    if (nseg == 0) {
        const int64_t base = (int64_t)s->ncomp * kp.tiles_u * kp.tiles_v;
        // about three blocks per CU (the VJP's register budget allows three)
        nseg = (int)std::max<int64_t>(1, std::min<int64_t>((target_blocks + base - 1) / base, (s->nw + 15) / 16));
    }
    nseg = std::min(nseg, s->nw);
    // segments start at multiples of the group length
    kp.seglen = ((s->nw + nseg - 1) / nseg + kGroup - 1) / kGroup * kGroup;
    kp.nseg = (s->nw + kp.seglen - 1) / kp.seglen;
    kp.nprim = s->nprim;
    kp.nclass = s->nclass;
    for (int c = 0; c < kMaxClasses; ++c) {
        kp.cls_node[c] = c < s->nclass ? s->classes[c].node : 0;
        kp.cls_sign[c] = c < s->nclass ? s->cls_sign[c] : 0.0;
        int wp = 0;
        if (c < s->nclass && s->classes[c].bounded) {
            wp = s->fields[s->classes[c].flo].idx >= 0 || s->fields[s->classes[c].fhi].idx >= 0;
        }
        kp.cls_wparam[c] = wp;
    }
    kp.nnode = s->nnode;
    kp.nlev = s->nlev;
    for (int k = 0; k < kMaxNodes; ++k) {
        kp.node_op[k] = s->node_op[k];
        kp.node_parent[k] = s->node_parent[k];
        kp.node_sign[k] = s->node_sign[k];
        kp.node_nm1[k] = s->node_nm1[k];
        kp.lev_node[k] = s->lev_node[k];
        kp.lev_q[k] = s->lev_q[k];
    }
    kp.eps_bg = s->eps_bg;
    kp.deps = s->eps_fg - s->eps_bg;
    for (int c = 0; c < kMaxComp; ++c) {
        const int cc = std::min(c, s->ncomp - 1);
        kp.uc[c] = s->d_lat + s->lat_off[cc][0];
        kp.uw[c] = s->d_lat + s->lat_off[cc][1];
        kp.vc[c] = s->d_lat + s->lat_off[cc][2];
        kp.vw[c] = s->d_lat + s->lat_off[cc][3];
    }
    kp.prims = s->d_prims;
    kp.cls = s->d_cls;
    kp.fref = s->d_fref;
    kp.consts = s->d_consts;
    kp.gseg = s->d_gseg;
    kp.grun = s->d_grun;
    kp.fval = s->d_fval[0];
    kp.bbox = s->d_bbox[0];
    kp.prec = s->d_prec[0];
    kp.ztab = s->d_ztab[0];
    kp.fval2 = s->d_fval[1];
    kp.bbox2 = s->d_bbox[1];
    kp.prec2 = s->d_prec[1];
    kp.ztab2 = s->d_ztab[s->static_w ? 0 : 1];
    kp.code = s->d_code[0];
    kp.code2 = s->d_code[s->static_w ? 0 : 1];
    kp.gcode = s->d_gcode[0];
    kp.gcode2 = s->d_gcode[s->static_w ? 0 : 1];
    return kp;
}

int64_t sg::staging_bytes(const sg_scene* s) {
    return 8 * std::max<int64_t>(1, s->nfield) + (16 + (int64_t)sizeof(PrimRec)) * s->nprim +
           28 * (int64_t)s->ncomp * s->nclass * s->nw + 4 * (int64_t)s->ncomp * ((s->nw + kGroup - 1) / kGroup) +
           16 * std::max<int64_t>(1, s->n_params);
}

static sg_status check_call(sg_ctx* ctx, sg_scene* s) {
    if (!ctx || !s) return fail(SG_E_INVALID, "NULL ctx or scene");
    if (s->ctx->device != ctx->device) return fail(SG_E_INVALID, "scene belongs to another device");
    HIP_OK(hipSetDevice(ctx->device));
    return SG_OK;
}

static sg_status finish_grad(sg_scene* s, double* grad, int grad_on_device, hipStream_t st) {
    if (grad_on_device || s->n_params == 0) return SG_OK;
    HIP_OK(hipMemcpyAsync(s->h_grad, s->d_grad, s->n_params * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    std::memcpy(grad, s->h_grad, s->n_params * sizeof(double));
    return SG_OK;
}

static hipError_t take_event(sg_scene* s, hipEvent_t* e) {
    if (!s->evpool.empty()) {
        *e = s->evpool.back();
        s->evpool.pop_back();
        return hipSuccess;
    }
    return hipEventCreate(e);
}

// Launches the column kernel; when tracing is on, a pair of events takes the
// kernel's start and end times (no dispatch gap counted).
static sg_status run_column(sg_scene* s, int mode, const KParams& kp, hipStream_t st) {
    if (!s->timing || (s->launches[mode & 7]++ % s->timing) != 0) {
        HIP_OK(launch_column(mode, s->tree, s->variant, kp, st));
        return SG_OK;
    }
    sg_scene::Rec r{mode, nullptr, nullptr};
    HIP_OK(take_event(s, &r.a));
    HIP_OK(take_event(s, &r.b));
    HIP_OK(launch_column(mode, s->tree, s->variant, kp, st, r.a, r.b));
    s->recs.push_back(r);
    return SG_OK;
}

// The F cache around one call: the planes and comparison buffers exist
// (allocated at first use, the first call's stage kernel forced to flag a
// change), the stage kernel compares the fields with those the planes were
// computed from, and the column kernel reads (no change) or writes the planes.
static sg_status fcache_prepare(sg_scene* s, StageParams& sp, KParams& kp, hipStream_t st) {
    const int64_t nuv = (int64_t)s->nu * s->nv;
    int force = 0;
    if (!s->d_fplane) {
        HIP_OK(hipMalloc((void**)&s->d_fplane, (size_t)s->ncomp * std::max(1, s->nclass) * nuv * sizeof(double)));
        HIP_OK(hipMalloc((void**)&s->d_fprev, std::max<int64_t>(1, s->nfield) * sizeof(double)));
        HIP_OK(hipMalloc((void**)&s->d_chg, 4 * sizeof(int32_t)));
        HIP_OK(launch_fill(reinterpret_cast<double*>(s->d_chg), 0.0, 2, st));     // all-zero bits
        force = 1;
    }
    // candidate lists for the rectangular split (the gradient's); a larger
    // split (set_launch) reallocates them, and the header then reads 0
    const KParams kr = column_params(s);
    const int64_t tiles = (int64_t)kr.ncomp * kr.tiles_u * kr.tiles_v;
    if (tiles > s->tlist_tiles) {
        hipFree(s->d_tlist);
        s->d_tlist = nullptr;
        s->tlist_tiles = 0;
        const int64_t words = 1 + tiles * (1 + kStageRec);
        HIP_OK(hipMalloc((void**)&s->d_tlist, ((words + 1) / 2) * 2 * sizeof(int32_t)));
        HIP_OK(launch_fill(reinterpret_cast<double*>(s->d_tlist), 0.0, 1, st));     // header 0: no lists
        s->tlist_tiles = tiles;
    }
    const int gen = s->fgen;
    s->fgen = (gen + 1) % 3;
    sp.fprev = s->d_fprev;
    sp.chg = s->d_chg;
    sp.gen = gen;
    sp.force = force;
    kp.fplane = s->d_fplane;
    kp.fprev = s->d_fprev;
    kp.chg = s->d_chg;
    kp.gen = gen;
    kp.nfield = (int32_t)s->nfield;
    kp.tlist = s->d_tlist;
    return SG_OK;
}

extern "C" sg_status sg_scene_set_timing(sg_scene* s, int enable) {
    if (!s) return fail(SG_E_INVALID, "NULL scene");
    std::lock_guard<std::mutex> lk(s->mu);
    HIP_OK(hipSetDevice(s->ctx->device));
    for (auto& r : s->recs) {
        HIP_OK(hipEventSynchronize(r.b));
        s->evpool.push_back(r.a);
        s->evpool.push_back(r.b);
    }
    s->recs.clear();
    if (enable < 0) return fail(SG_E_INVALID, "sg_scene_set_timing: negative period");
    s->timing = enable;
    for (auto& n : s->launches) n = 0;
    return SG_OK;
}

extern "C" sg_status sg_scene_kernel_time(sg_scene* s, int mode, double* total_ms, int64_t* launches) {
    if (!s || !total_ms || !launches) return fail(SG_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    HIP_OK(hipSetDevice(s->ctx->device));
    double t = 0.0;
    int64_t n = 0;
    for (auto& r : s->recs) {
        if (r.mode != mode) continue;
        HIP_OK(hipEventSynchronize(r.b));
        float ms = 0.0f;
        HIP_OK(hipEventElapsedTime(&ms, r.a, r.b));
        t += ms;
        ++n;
    }
    *total_ms = t;
    *launches = n;
    return SG_OK;
}

extern "C" sg_status eps_build(sg_ctx* ctx, sg_scene* s, const double* p, int p_on_device, float* eps, void* stream) {
    sg_status rc = check_call(ctx, s);
    if (rc != SG_OK) return rc;
    if (!eps) return fail(SG_E_INVALID, "eps is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    hipStream_t st = (hipStream_t)stream;
    const double* dp;
    if ((rc = stage_p(s, p, p_on_device, st, &dp)) != SG_OK) return rc;
    StageParams sp = stage_params(s, dp);
    // eps_build writes 4 B per sample against the VJP's 16 B read: on short
    // columns each segment repeats the tile's prologue for a quarter of the
    // VJP's bytes, so it aims at half the VJP's blocks (blazed grating, with
    // the blocks in segment-slowest order: 13.7 us at 384 blocks, 14.5 us at
    // 960).  Linear tiles: every wavefront stores 64 consecutive floats per step, so
    // whole 128-byte lines leave with the non-temporal stores (a 128 x 2 tile
    // on a 600-wide grid writes 256-byte runs that straddle line boundaries;
    // measured on the taper: 71.6 -> 40.2 us)
    KParams kp = column_params(s, 384, true);
    if (s->fcache && (rc = fcache_prepare(s, sp, kp, st)) != SG_OK) return rc;
    HIP_OK(launch_stage(sp, 1, st));
    kp.out = eps;
    return run_column(s, MODE_EPS, kp, st);
}

// Device buffers of one call's staging (scene-owned, or carved from the
// scratch array by eps_grad_vjp_noalloc).
struct Staging {
    double* fval = nullptr;
    float4* bbox = nullptr;
    PrimRec* prec = nullptr;
    double* ztab = nullptr;              // only when the extrusion tables depend on p
    uint32_t* code = nullptr;
    uint32_t* gcode = nullptr;
    double* gspread = nullptr;           // spread accumulation
    unsigned long long* fx = nullptr;    // deterministic reduction
};

// Lays out one VJP call's staging at base; returns the bytes it needs (each
// table aligned to 256 bytes).  base == nullptr only measures.
static int64_t scratch_layout(const sg_scene* s, bool det, bool spread, char* base, Staging* st) {
    int64_t off = 0;
    auto take = [&](int64_t bytes) -> char* {
        char* q = base ? base + off : nullptr;
        off += (std::max<int64_t>(bytes, 1) + 255) / 256 * 256;
        return q;
    };
    const int64_t n = std::max<int64_t>(1, s->n_params);
    st->fval = (double*)take(8 * std::max<int64_t>(1, s->nfield));
    st->bbox = (float4*)take((int64_t)sizeof(float4) * s->nprim);
    st->prec = (PrimRec*)take((int64_t)sizeof(PrimRec) * s->nprim);
    if (!s->static_w) {
        st->ztab = (double*)take(24 * (int64_t)s->ncomp * s->nclass * s->nw);
        st->code = (uint32_t*)take(4 * (int64_t)s->ncomp * s->nw);
        st->gcode = (uint32_t*)take(4 * (int64_t)s->ncomp * ((s->nw + kGroup - 1) / kGroup));
    }
    if (spread) st->gspread = (double*)take(8 * (int64_t)kGradSpread * n);
    if (det) st->fx = (unsigned long long*)take(8 * (3 * n + 1));
    return off;
}

static sg_status vjp_common(sg_ctx* ctx, sg_scene* s, const double* p, int p_on_device, int mode,
                            const void* const* e_fwd, const void* const* e_adj, double omega, const float* geps,
                            double* grad, int grad_on_device, void* stream, bool noalloc = false) {
    sg_status rc = check_call(ctx, s);
    if (rc != SG_OK) return rc;
    if (!grad && s->n_params > 0) return fail(SG_E_INVALID, "grad is NULL");
    const bool fields = mode == MODE_VJP_FIELDS || mode == MODE_VJP_SPARSE;
    if (fields) {
        if (!e_fwd || !e_adj) return fail(SG_E_INVALID, "field pointer arrays are NULL");
        for (int c = 0; c < s->ncomp; ++c)
            if (!e_fwd[c] || !e_adj[c]) return fail(SG_E_INVALID, "field plane %d is NULL", c);
        if (!std::isfinite(omega)) return fail(SG_E_INVALID, "omega not finite");
    } else if (!geps) {
        return fail(SG_E_INVALID, "grad_eps is NULL");
    }
    std::lock_guard<std::mutex> lk(s->mu);
    hipStream_t st = (hipStream_t)stream;
    const bool det = s->deterministic && s->n_params > 0;
    const bool spread = !det && s->spread && s->n_params > 0;
    Staging stg;
    if (noalloc) {
        // every per-call table in the scratch array: no allocation on any path
        const int64_t need = scratch_layout(s, det, spread, (char*)ctx->scratch, &stg);
        if (need > kScratchBytes)
            return fail(SG_E_TOO_LARGE, "eps_grad_vjp_noalloc: the scene's staging needs %lld bytes, the scratch holds "
                        "%lld", (long long)need, (long long)kScratchBytes);
    } else {
        stg.fval = s->d_fval[0];
        stg.bbox = s->d_bbox[0];
        stg.prec = s->d_prec[0];
        if (!s->static_w) {
            stg.ztab = s->d_ztab[0];
            stg.code = s->d_code[0];
            stg.gcode = s->d_gcode[0];
        }
        stg.gspread = s->d_gspread;
        if (det) {
            if (!s->d_fx) HIP_OK(hipMalloc((void**)&s->d_fx, (3 * s->n_params + 1) * sizeof(unsigned long long)));
            stg.fx = s->d_fx;
        }
    }
    const double* dp;
    if ((rc = stage_p(s, p, p_on_device, st, &dp)) != SG_OK) return rc;
    double* g = grad_on_device ? grad : s->d_grad;
    StageParams sp = stage_params(s, dp);
    sp.fval[0] = stg.fval;
    sp.bbox[0] = stg.bbox;
    sp.prec[0] = stg.prec;
    if (!s->static_w) {
        sp.ztab[0] = stg.ztab;
        sp.code[0] = stg.code;
        sp.gcode[0] = stg.gcode;
    }
    sp.zero_ptr = g;
    sp.zero_n = s->n_params;
    KParams kp = column_params(s);
    if (s->fcache && !noalloc && mode != MODE_VJP_SPARSE && (rc = fcache_prepare(s, sp, kp, st)) != SG_OK) return rc;
    HIP_OK(launch_stage(sp, 1, st));
    kp.fval = stg.fval;
    kp.bbox = stg.bbox;
    kp.prec = stg.prec;
    if (!s->static_w) {
        kp.ztab = stg.ztab;
        kp.code = stg.code;
        kp.gcode = stg.gcode;
    }
    kp.grad = g;
    if (mode == MODE_VJP_SPARSE) {
        // its segments split only the steps where some class is nonzero, and
        // each segment's block repeats the tile's in-plane work: a quarter of
        // the dense split (unless the caller fixed it)
        if (s->nseg == 0) {
            kp.nseg = (kp.nseg + 3) / 4;
            kp.seglen = ((s->nw + kp.nseg - 1) / kp.nseg + kGroup - 1) / kGroup * kGroup;
            kp.nseg = (s->nw + kp.seglen - 1) / kp.seglen;
        }
        if (!s->d_nread) HIP_OK(hipMalloc((void**)&s->d_nread, kReadSlots * sizeof(unsigned long long)));
        HIP_OK(launch_fill(reinterpret_cast<double*>(s->d_nread), 0.0, kReadSlots, st));
        kp.nread = s->d_nread;
    }
    // the spread copies and the fixed-point accumulators start at zero (a
    // fill kernel: they hold the previous call's sums)
    if (spread) {
        HIP_OK(launch_fill(stg.gspread, 0.0, (int64_t)kGradSpread * s->n_params, st));
        kp.grad = stg.gspread;
        kp.gstride = s->n_params;
    }
    if (det) {
        const int64_t words = 3 * s->n_params + 1;
        HIP_OK(launch_fill(reinterpret_cast<double*>(stg.fx), 0.0, words, st));   // all-zero bits
        kp.fx = stg.fx;
        kp.fx_n = s->n_params;
    }
    if (fields) {
        for (int c = 0; c < kMaxComp; ++c) {
            const int cc = std::min(c, s->ncomp - 1);
            kp.ef[c] = (const float2*)e_fwd[cc];
            kp.ea[c] = (const float2*)e_adj[cc];
        }
        kp.two_omega = (float)(2.0 * omega);
    } else {
        kp.geps = geps;
    }
    if (noalloc) {
        HIP_OK(launch_column(mode, s->tree, s->variant, kp, st));     // untraced: tracing creates events
    } else if ((rc = run_column(s, mode, kp, st)) != SG_OK) {
        return rc;
    }
    if (det) HIP_OK(launch_fx_finish(stg.fx, s->n_params, g, st));
    if (spread) HIP_OK(launch_spread_finish(stg.gspread, s->n_params, g, st));
    return finish_grad(s, grad, grad_on_device, st);
}

extern "C" sg_status sg_scene_set_deterministic(sg_scene* s, int enable) {
    if (!s) return fail(SG_E_INVALID, "NULL scene");
    std::lock_guard<std::mutex> lk(s->mu);
    s->deterministic = enable != 0;
    return SG_OK;
}

extern "C" sg_status eps_grad_vjp(sg_ctx* ctx, sg_scene* s, const double* p, int p_on_device, const void* const* e_fwd,
                                  const void* const* e_adj, double omega, double* grad, int grad_on_device,
                                  void* stream) {
    return vjp_common(ctx, s, p, p_on_device, MODE_VJP_FIELDS, e_fwd, e_adj, omega, nullptr, grad, grad_on_device,
                      stream);
}

extern "C" sg_status eps_grad_vjp_noalloc(sg_ctx* ctx, sg_scene* s, const double* p, int p_on_device,
                                          const void* const* e_fwd, const void* const* e_adj, double omega,
                                          double* grad, int grad_on_device, void* stream) {
    return vjp_common(ctx, s, p, p_on_device, MODE_VJP_FIELDS, e_fwd, e_adj, omega, nullptr, grad, grad_on_device,
                      stream, true);
}

extern "C" sg_status eps_grad_vjp_sparse(sg_ctx* ctx, sg_scene* s, const double* p, int p_on_device,
                                         const void* const* e_fwd, const void* const* e_adj, double omega,
                                         double* grad, int grad_on_device, void* stream) {
    return vjp_common(ctx, s, p, p_on_device, MODE_VJP_SPARSE, e_fwd, e_adj, omega, nullptr, grad, grad_on_device,
                      stream);
}

extern "C" sg_status sg_scene_sparse_reads(sg_scene* s, int64_t* pairs) {
    if (!s || !pairs) return fail(SG_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    HIP_OK(hipSetDevice(s->ctx->device));
    unsigned long long v[kReadSlots] = {};
    if (s->d_nread) HIP_OK(hipMemcpy(v, s->d_nread, sizeof(v), hipMemcpyDeviceToHost));
    int64_t n = 0;
    for (int i = 0; i < kReadSlots; ++i) n += (int64_t)v[i];
    *pairs = n;
    return SG_OK;
}

extern "C" sg_status eps_grad_vjp_geps(sg_ctx* ctx, sg_scene* s, const double* p, int p_on_device,
                                       const float* grad_eps, double* grad, int grad_on_device, void* stream) {
    return vjp_common(ctx, s, p, p_on_device, MODE_VJP_GEPS, nullptr, nullptr, 0.0, grad_eps, grad, grad_on_device,
                      stream);
}

static sg_status fd_common(sg_ctx* ctx, sg_scene* s, const double* p, int p_on_device, const void* const* e_fwd,
                           const void* const* e_adj, double omega, double h, int scheme, double* grad,
                           int grad_on_device, void* stream, bool sparse) {
    sg_status rc = check_call(ctx, s);
    if (rc != SG_OK) return rc;
    if (!grad && s->n_params > 0) return fail(SG_E_INVALID, "grad is NULL");
    if (!e_fwd || !e_adj) return fail(SG_E_INVALID, "field pointer arrays are NULL");
    for (int c = 0; c < s->ncomp; ++c)
        if (!e_fwd[c] || !e_adj[c]) return fail(SG_E_INVALID, "field plane %d is NULL", c);
    if (!(h > 0.0) || !std::isfinite(h)) return fail(SG_E_INVALID, "h must be > 0");
    if (scheme != SG_FD_CENTRAL && scheme != SG_FD_FORWARD) return fail(SG_E_INVALID, "unknown FD scheme");
    std::lock_guard<std::mutex> lk(s->mu);
    hipStream_t st = (hipStream_t)stream;
    const int64_t total = (int64_t)s->ncomp * s->plane;
    for (int v = 0; v < (sparse ? 1 : 2); ++v)
        if (!s->d_work[v]) HIP_OK(hipMalloc((void**)&s->d_work[v], total * sizeof(float) + 64));
    const double* dp;
    if ((rc = stage_p(s, p, p_on_device, st, &dp)) != SG_OK) return rc;
    double* g = grad_on_device ? grad : s->d_grad;
    HIP_OK(launch_fill(g, 0.0, std::max<int64_t>(1, s->n_params), st));
    const float2* ef[3];
    const float2* ea[3];
    for (int c = 0; c < 3; ++c) {
        const int cc = std::min(c, s->ncomp - 1);
        ef[c] = (const float2*)e_fwd[cc];
        ea[c] = (const float2*)e_adj[cc];
    }
    HIP_OK(launch_gplane(ef, ea, s->ncomp, s->plane, (float)(2.0 * omega), s->d_work[0], st));
    KParams kp = column_params(s);
    const double scale = scheme == SG_FD_CENTRAL ? 1.0 / (2.0 * h) : 1.0 / h;
    if (sparse) {
        kp.geps = s->d_work[0];
        kp.grad = g;
        kp.kprim_off = s->d_kprim_off;
        kp.kprim = s->d_kprim;
        kp.fd_scale = scale;
        if (s->nseg == 0) {     // as the sparse VJP: the segments split only the live steps
            kp.nseg = (kp.nseg + 3) / 4;
            kp.seglen = ((s->nw + kp.nseg - 1) / kp.nseg + kGroup - 1) / kGroup * kGroup;
            kp.nseg = (s->nw + kp.seglen - 1) / kp.seglen;
        }
    } else {
        kp.out = s->d_work[1];
    }
    for (int64_t k = 0; k < s->n_params; ++k) {
        // (sparse) a parameter no field references has a zero derivative
        if (sparse && s->kprim_off[k + 1] == s->kprim_off[k] && !s->k_wbound[k]) continue;
        StageParams sp = stage_params(s, dp);
        sp.pert_idx = k;
        sp.delta[0] = h;
        sp.delta[1] = scheme == SG_FD_CENTRAL ? -h : 0.0;
        HIP_OK(launch_stage(sp, 2, st));
        if (sparse) {
            kp.fd_k = (int32_t)k;
            kp.fd_all = s->k_wbound[k];
            if ((rc = run_column(s, MODE_FD_SPARSE, kp, st)) != SG_OK) return rc;
        } else {
            if ((rc = run_column(s, MODE_FD, kp, st)) != SG_OK) return rc;
            HIP_OK(launch_dot(s->d_work[0], s->d_work[1], total, scale, g + k, st));
        }
    }
    return finish_grad(s, grad, grad_on_device, st);
}

extern "C" sg_status eps_grad_fd(sg_ctx* ctx, sg_scene* s, const double* p, int p_on_device, const void* const* e_fwd,
                                 const void* const* e_adj, double omega, double h, int scheme, double* grad,
                                 int grad_on_device, void* stream) {
    return fd_common(ctx, s, p, p_on_device, e_fwd, e_adj, omega, h, scheme, grad, grad_on_device, stream, false);
}

extern "C" sg_status eps_grad_fd_sparse(sg_ctx* ctx, sg_scene* s, const double* p, int p_on_device,
                                        const void* const* e_fwd, const void* const* e_adj, double omega, double h,
                                        int scheme, double* grad, int grad_on_device, void* stream) {
    return fd_common(ctx, s, p, p_on_device, e_fwd, e_adj, omega, h, scheme, grad, grad_on_device, stream, true);
}

// ------------------------------------------------------------------ utilities
extern "C" sg_status sg_util_copy(void* dst, const void* src, int64_t bytes, void* stream) {
    if (!dst || !src || bytes < 0 || (bytes % 16) != 0) return fail(SG_E_INVALID, "sg_util_copy: bad arguments");
    HIP_OK(launch_copy(dst, src, bytes, (hipStream_t)stream));
    return SG_OK;
}

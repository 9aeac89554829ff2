// Host-side internals shared by the C-ABI entry points (sg_api.hip) and the
// serving runtime (sg_serve.hip): error state, context and compiled scene.
#pragma once

#include <mutex>
#include <string>
#include <vector>

#include "sg_internal.h"

namespace sg {

sg_status fail(sg_status code, const char* fmt, ...);

}  // namespace sg

#define HIP_OK(call)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess) return sg::fail(SG_E_DEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

struct sg_ctx {
    int device;
    void* scratch = nullptr;    // device address of this device's copy of the allocation-free scratch array
};

struct sg_scene {
    sg_ctx* ctx = nullptr;
    int dim = 0, ncomp = 0, comp_axis[3] = {0, 0, 0};
    int64_t n[3] = {0, 0, 0};
    int64_t n_params = 0;
    int64_t nfield = 0;
    double eps_bg = 0, eps_fg = 0;
    int col = 2;                      // column axis: 1 (y) or 2 (z)
    int axis_v = 1;
    int nu = 0, nv = 0, nw = 0;
    int64_t sv = 0, sw = 0, plane = 0;
    int nprim = 0, nclass = 0, ncls_pad = 1;
    int variant = sg::VAR_ALL;
    int tree = sg::TR_GEN8;
    // the general composition program (see KParams)
    int nnode = 0, nlev = 0;
    int node_op[sg::kMaxNodes] = {};
    int node_parent[sg::kMaxNodes] = {};
    int lev_node[sg::kMaxNodes] = {};
    double node_sign[sg::kMaxNodes] = {};
    double node_nm1[sg::kMaxNodes] = {};
    double lev_q[sg::kMaxNodes] = {};
    std::vector<double> cls_sign;
    std::vector<sg::DevClass> classes;
    std::vector<sg_field> fields;
    int block_x = 0, nseg = 0;        // 0: automatic
    bool linear_tiles = true;         // eps_build on linear tiles (SG_EPS_RECT_TILES=1 at creation: off)
    // device tables
    double* d_lat = nullptr;          // per component: uc uw vc vw wc ww
    int64_t lat_off[sg::kMaxComp][6] = {};
    sg_field* d_fref = nullptr;
    sg::DevPrim* d_prims = nullptr;
    sg::DevClass* d_cls = nullptr;
    double* d_consts = nullptr;
    sg::GSeg* d_gseg = nullptr;
    double* d_p = nullptr;
    double* d_fval[2] = {nullptr, nullptr};
    float4* d_bbox[2] = {nullptr, nullptr};
    sg::PrimRec* d_prec[2] = {nullptr, nullptr};
    double* d_ztab[2] = {nullptr, nullptr};
    uint32_t* d_code[2] = {nullptr, nullptr};   // column-step codes
    uint32_t* d_gcode[2] = {nullptr, nullptr};  // group codes
    int32_t* d_grun = nullptr;                  // static codes only: ends of the runs of equal group codes
    double* d_grad = nullptr;
    // no extrusion bound references a parameter: the extrusion tables and
    // step / group codes (index 0) are computed once, at scene creation, and
    // serve every call and both FD evaluation points
    bool static_w = false;
    float* d_work[2] = {nullptr, nullptr};
    unsigned long long* d_nread = nullptr;   // sparse VJP: (sample, step) pairs read
    bool deterministic = false;              // fixed-point (order-independent) VJP sums
    unsigned long long* d_fx = nullptr;      // their accumulators: 3 n + 1 words
    // parameters shared by many blocks (one referenced by many primitives, or
    // a sine-series term): the VJP spreads its atomics over kGradSpread copies
    bool spread = false;
    double* d_gspread = nullptr;             // kGradSpread x n
    // F cache (eps_build, eps_grad_vjp, eps_grad_vjp_geps): the in-plane
    // sums of every sample (ncomp x nclass x nu nv FP64) and the fields they
    // were computed from, allocated at first use; the stage kernel of call
    // `fgen` compares the fields and flags d_chg[fgen % 3]
    bool fcache = true;                      // by feature set; SG_F_CACHE=0 / 1 at creation: off / on
    double* d_fplane = nullptr;
    double* d_fprev = nullptr;
    int32_t* d_chg = nullptr;
    int32_t fgen = 0;
    int32_t* d_tlist = nullptr;              // the tiles' candidate lists (room for tlist_tiles tiles)
    int64_t tlist_tiles = 0;
    // sparse FD: the primitives (device order) whose fields reference each
    // parameter, CSR; and the parameters an extrusion bound references
    std::vector<int32_t> kprim_off, kprim;
    std::vector<char> k_wbound;
    int32_t* d_kprim_off = nullptr;
    int32_t* d_kprim = nullptr;
    double* h_p = nullptr;            // pinned staging
    double* h_grad = nullptr;
    hipEvent_t p_evt = nullptr;
    bool p_evt_pending = false;
    // tracing: events around the column-kernel launches
    int timing = 0;                   // record every timing-th launch of each kind (0: off)
    int64_t launches[8] = {};         // column-kernel launches per kind since timing was set
    struct Rec {
        int mode;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> evpool;
    std::mutex mu;
};

namespace sg {
// launch parameters of a scene's kernels, pointing at its own staging buffers
StageParams stage_params(sg_scene* s, const double* dp);
// target_blocks: the block count the automatic column split aims for;
// linear: linear tiles where the scene's rows are contiguous
KParams column_params(sg_scene* s, int64_t target_blocks = 768, bool linear = false);
// bytes of device staging one gradient evaluation of the scene needs
int64_t staging_bytes(const sg_scene* s);
}  // namespace sg

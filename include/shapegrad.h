/*
 * shapegrad.h -- C ABI of the MI355X shape-parameter gradient library.
 *
 * The library implements steps 2 and 5 of the adjoint inverse-design loop
 * (Sec. "Background on photonic inverse design and the adjoint method"):
 *   step 2: design vector v (here p, n FP64 values) -> permittivity eps(p) on a
 *           rectilinear grid, built from AutoDiffGeo primitives (Sec.
 *           "AutoDiffGeo", Tab. autodiffgeo) rasterized to fill fractions with
 *           sigma_k (Tab. nonlinearfunctions), combined by eq:union,
 *           eq:intersection and difference, and scaled to two materials;
 *   step 5: the adjoint gradient of eq:1 (epsilon term),
 *           grad_k = sum over components c and samples j of
 *                    Re(c0 * E_cj * Eadj_cj) * d eps_cj / d p_k,  c0 = -2i*omega,
 *           computed in reverse mode (eq:AD, eq:jaceps) without forming the
 *           Jacobian, or by finite differences (the paper's baseline).
 * The fields E and E_adj are given inputs (Sec. "Background": the simulators
 * are out of scope).
 *
 * Conventions shared by every call
 *   - Every function returns sg_status: SG_OK (0), SG_EAGAIN (1, serving only)
 *     or a negative error.  Nothing throws across the ABI and nothing exits.
 *     sg_last_error() returns a thread-local message for the last failure on
 *     the calling thread (valid until that thread's next call).
 *   - Planes are FP32 (eps, dF/deps) or complex64 (interleaved re, im) arrays
 *     of shape [Nz][Ny][Nx], x fastest; a component set is C planes.  All plane
 *     pointers are device memory owned by the caller.
 *   - Component c of a set is the field component along axis comp_axis[c];
 *     it samples the material at the cell center along its own axis and at the
 *     cell's lower node along the other axes (staggered Yee positions).
 *   - p: n_params FP64, on the host (p_on_device = 0, copied before the call
 *     returns) or on the device (1, read by the call's stream work).
 *   - grad: n_params FP64, overwritten.  On the host (grad_on_device = 0) the
 *     call blocks until the result is there; on the device it is asynchronous.
 *   - stream: a hipStream_t (NULL = the default stream).  Device work is
 *     ordered on it.  Calls on one scene must be ordered on one stream (a
 *     scene owns its staging buffers); use one scene per concurrent stream.
 *   - Invalid input (null pointer, size or index out of range, NaN in p,
 *     unknown type) is rejected on the host before any launch (SG_E_INVALID).
 *     HIP failures return SG_E_DEVICE on this call or the next.
 */
#ifndef SHAPEGRAD_H
#define SHAPEGRAD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t sg_status;
enum {
    SG_OK = 0,
    SG_EAGAIN = 1,
    SG_E_INVALID = -1,
    SG_E_NOMEM = -2,
    SG_E_TOO_LARGE = -3,
    SG_E_DEVICE = -4,
    SG_E_CANCELLED = -5,
    SG_E_TIMEOUT = -6,
    SG_E_UNSUPPORTED = -7
};

/* Primitive types (Tab. autodiffgeo).  Field order per type:
 *   SG_PRIM_BOX     x0 x1 y0 y1 z0 z1           RectdD = product of Rect1D per bounded axis
 *                                               sigma[0..2] = x, y, z
 *   SG_PRIM_ELLIPSE x0 y0 r z0 z1               Circ2D with aspect transform:
 *                                               sigma_k(r - rho), rho = |((x-x0)/ax, (y-y0)/ay)|
 *                                               consts: ax ay; sigma[0] boundary (FIXED k), sigma[2] z
 *   SG_PRIM_POLY    x_1..x_N y_1..y_N z0 z1     Poly2D: product of Step2D over the edges of a
 *                                               convex counter-clockwise polygon (inward normals)
 *                                               sigma[0] boundary (FIXED k), sigma[2] z
 *   SG_PRIM_GCART   xs xe y+_1..y+_M y-_1..y-_M z0 z1
 *                                               two-sided GeneralCartesian2D:
 *                                               Rect1D(x; xs, xe) sigma_k(f+(x) - y) sigma_k(y - f-(x))
 *                                               with f+- piecewise linear through (x_j, y+-_j),
 *                                               constant beyond the end vertices;
 *                                               consts: x_1 < ... < x_M; sigma[0] x-range,
 *                                               sigma[1] y boundary, sigma[2] z
 *   SG_PRIM_POLAR   x0 y0 R0 c_1..c_N s_1..s_N z0 z1   (nvert = N, 1 <= N <= 29)
 *                                               GeneralPolar2D with the Fourier radius of
 *                                               eq:PSGCboundary: sigma_k(R(theta) - r), r and theta
 *                                               the polar coordinates about (x0, y0),
 *                                               R = R0 + sum_n c_n cos(n theta + pi) + s_n sin(n theta + pi);
 *                                               sigma[0] boundary (FIXED k), sigma[2] z
 *   SG_PRIM_POLAR2D x0 y0 R delta z0 z1         (nvert = alpha, 1 <= alpha <= 64)
 *                                               Polar2D: sigma_k(R (1 + delta cos(alpha theta)) - r),
 *                                               r and theta the polar coordinates about (x0, y0)
 *                                               (theta over the full turn, so alpha is an integer);
 *                                               sigma[0] boundary (FIXED k), sigma[2] z
 *   SG_PRIM_SERIES  xs xe v_1..v_K z0 z1        (nvert = K, 1 <= K <= 4096)
 *                                               two-sided boundary with the sine series of
 *                                               eq:taper_boundary: Rect1D(x; xs, xe)
 *                                               sigma_k(f(x) - (y - yc)) sigma_k(f(x) + (y - yc)),
 *                                               f = w_in/2 + (w_out - w_in)/2 (x - x0)/L
 *                                                 + env(x) sum_i v_i sin(i pi (x - x0)/L),
 *                                               env = 0.1 + 0.45 (1 - cos(2 pi (x - x0)/L));
 *                                               consts: x0 L w_in w_out yc; sigma[0] x-range,
 *                                               sigma[1] y boundary, sigma[2] z
 * z0 z1 are the extrusion along z (Rect1D in z), used when bounded[2] != 0.
 * In 2D scenes (dim = 2) nothing may be bounded along z. */
enum { SG_PRIM_BOX = 0, SG_PRIM_ELLIPSE = 1, SG_PRIM_POLY = 2, SG_PRIM_GCART = 3, SG_PRIM_POLAR = 4,
       SG_PRIM_SERIES = 5, SG_PRIM_POLAR2D = 6 };

/* sigma_k kinds (Tab. nonlinearfunctions).  sigmoid and erf are taken as exactly
 * 0 / 1 beyond |k x| = 24 / 6 (tails below 4e-11 / 2e-17). */
enum { SG_SIGMA_SIGMOID = 0, SG_SIGMA_ERF = 1, SG_SIGMA_SIN = 2, SG_SIGMA_LINEAR = 3, SG_SIGMA_QUADRATIC = 4 };
/* k modes: LOCAL k = k / (sample width along the argument's axis); FIXED k as given (1/um). */
enum { SG_K_LOCAL = 0, SG_K_FIXED = 1 };
/* op-tree nodes: union min{1, sum} (eq:union), intersection max{N-1, sum} - (N-1)
 * (eq:intersection), difference max{0, a - b} (exactly two operands), and the
 * non-binary union of Alg. cap (Sec. "Non-binary material systems"), root
 * only: children are K >= 2 material sets (each a union / intersection node or
 * one primitive) with levels eps^1 <= ... <= eps^K relative to the background
 * (consts[aux .. aux + K), the top one equal to eps_fg - eps_bg);
 * s = v_1, s = min{1, (eps^{k-1} / eps^k) s + v_k} for k = 2..K, eps = eps_bg + eps^K s. */
enum { SG_OP_UNION = 0, SG_OP_INTERSECTION = 1, SG_OP_DIFFERENCE = 2, SG_OP_LEVELS = 3 };
/* finite-difference schemes for eps_grad_fd */
enum { SG_FD_CENTRAL = 0, SG_FD_FORWARD = 1 };

typedef struct sg_field { double a; double b; int64_t idx; } sg_field;   /* a + b * p[idx]; idx < 0: a */
typedef struct sg_sigma { int32_t kind; int32_t kmode; double k; } sg_sigma;

typedef struct sg_prim_desc {
    int32_t type;
    int32_t nvert;        /* POLY: N (>= 3); GCART: M (>= 2); else 0 */
    int32_t field_off;    /* first field in sg_scene_desc.fields */
    int32_t nfield;       /* BOX 6, ELLIPSE 5, POLY 2N+2, GCART 2M+4 */
    int32_t const_off;    /* first constant in sg_scene_desc.consts */
    int32_t nconst;       /* ELLIPSE 2, GCART M, else 0 */
    int32_t bounded[3];   /* BOX: per axis; others: [2] = extruded along z */
    int32_t pad;
    sg_sigma sigma[3];
} sg_prim_desc;

typedef struct sg_node_desc {
    int32_t op;
    int32_t nchild;
    int32_t child_off;    /* into sg_scene_desc.children */
    int32_t aux;          /* SG_OP_LEVELS: first of its nchild level values in consts */
} sg_node_desc;

typedef struct sg_scene_desc {
    int32_t dim;              /* 2 or 3 */
    int32_t ncomp;            /* 1..3 */
    int32_t comp_axis[3];     /* 0 = x, 1 = y, 2 = z */
    int32_t pad0;
    int64_t n[3];             /* Nx, Ny, Nz cells (Nz = 1 when dim = 2) */
    const double* nodes[3];   /* node coordinates in um, n[a] + 1 each, increasing */
    double eps_bg;            /* background permittivity */
    double eps_fg;            /* shape permittivity */
    int64_t n_params;
    int32_t nprim, nfield, nconst, nnode, nchild, pad1;
    const sg_prim_desc* prims;
    const sg_field* fields;
    const double* consts;
    const sg_node_desc* nodes_op;   /* postfix order, root last */
    const int32_t* children;        /* >= 0: primitive; < 0: node -(c + 1), earlier in the list */
} sg_scene_desc;

typedef struct sg_ctx sg_ctx;
typedef struct sg_scene sg_scene;

/* Context on one HIP device.  Thread-safe for distinct scenes. */
sg_status sg_ctx_create(int hip_device, sg_ctx** out);
void sg_ctx_destroy(sg_ctx* ctx);
const char* sg_last_error(void);

/* Compile a scene description (copied; the caller's arrays may be freed after
 * the call) into device tables.  Op trees of any shape and depth (eq:eps:
 * nested unions, intersections and differences, a levels node as the root)
 * with at most 6 op nodes (a levels root turns each primitive among its
 * material sets into a node of its own) and at most 8 extrusion classes (the
 * primitives that are children of one node with the same sign there and the
 * same factor along the column axis form one class); larger trees return
 * SG_E_UNSUPPORTED.  Every node must lie below the root and every primitive
 * may appear once. */
sg_status sg_scene_create(sg_ctx* ctx, const sg_scene_desc* desc, sg_scene** out);
void sg_scene_destroy(sg_scene* scene);
sg_status sg_scene_info(const sg_scene* scene, int64_t* n_params, int32_t* ncomp, int64_t dims[3]);
/* Deterministic reduction for eps_grad_vjp, eps_grad_vjp_sparse and
 * eps_grad_vjp_geps: the sum over samples of eq. (1) (default: off, or on
 * when the environment variable SG_DETERMINISTIC is a nonzero integer at
 * scene creation).  Each wavefront's FP64 contribution is rounded down to a
 * multiple of 2^-64 and added exactly, as 32-bit limbs in 64-bit integer
 * accumulators (3 n + 1 words the scene owns), which a last kernel turns back
 * into FP64; integer sums do not depend on the order of the additions, so
 * repeated calls with the same inputs and launch shape give bitwise-equal
 * gradients.  It agrees with the atomic mode to about 2^-64 per contribution
 * plus the FP64 rounding of the atomic sums.  A contribution of magnitude
 * >= 2^31 (or NaN) makes every entry of the gradient NaN.  A serving session
 * takes the scene's setting when it opens (serve_open_session); the FD entry
 * points always use atomics. */
sg_status sg_scene_set_deterministic(sg_scene* scene, int enable);

/* Launch shape override: block width in x (16, 32, 64, 128 or 256 samples; the
 * block holds 256 samples) and the number of segments each sample column is
 * split into (>= 1).  0 keeps the library's choice. */
sg_status sg_scene_set_launch(sg_scene* scene, int32_t block_x, int32_t col_segments);

/* Step 2 (Sec. "Background"; eq:eps): eps[C][Nz][Ny][Nx] FP32 = eps_bg +
 * (eps_fg - eps_bg) * s(p), with s composed in FP64 and rounded once. */
sg_status eps_build(sg_ctx* ctx, sg_scene* scene, const double* p, int p_on_device,
                    float* eps, void* stream);

/* Step 5, fused (eq:1, eq:AD): e_fwd and e_adj are arrays of C device pointers
 * to complex64 planes.  grad_k = sum_c sum_j 2*omega*Im(E_cj Eadj_cj) d eps_cj/d p_k
 * (no conjugation).  The mu / H term of eq:1 has the same form: call this with
 * a scene describing mu and the H, H_adj planes, and add the two gradients. */
sg_status eps_grad_vjp(sg_ctx* ctx, sg_scene* scene, const double* p, int p_on_device,
                       const void* const* e_fwd, const void* const* e_adj, double omega,
                       double* grad, int grad_on_device, void* stream);

/* eps_grad_vjp for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): same
 * arguments and result (up to the order of the floating-point sums; bitwise
 * the same in deterministic mode), but the call allocates nothing.  Its
 * per-call staging (resolved fields, support boxes, primitive records, the
 * extrusion tables when they depend on p, spread gradient copies or
 * fixed-point accumulators) lives in a 4 MiB device array that the library
 * holds on every device it runs on until the process ends, and that every
 * such call on the device shares: calls that overlap on one device (on
 * different streams or threads) race and give wrong results.  Scenes whose
 * staging exceeds 4 MiB return SG_E_TOO_LARGE before any launch.  p and grad
 * on the host use the scene's pinned staging (allocated by sg_scene_create).
 * Not traced by sg_scene_set_timing. */
sg_status eps_grad_vjp_noalloc(sg_ctx* ctx, sg_scene* scene, const double* p, int p_on_device,
                               const void* const* e_fwd, const void* const* e_adj, double omega,
                               double* grad, int grad_on_device, void* stream);

/* Step 5, sparse form (Sec. "Single-polarization blazed grating coupler in 2D",
 * item (iv): restrict the material Jacobian to where shapes are perturbed;
 * Sec. "Discussion and Conclusion": track its nonzero entries along shape
 * boundaries).  Same arguments and result as eps_grad_vjp, but the fields are
 * read only where d eps / d p can be nonzero: at samples where some
 * primitive's in-plane sigma argument lies inside its support (with the
 * primitive's other factors nonzero), and on column steps where some
 * extrusion class is nonzero.  Entries equal eps_grad_vjp's up to the order of
 * the floating-point sums.  Scenes whose extrusion bounds carry parameters
 * read every sample (those partials reach wherever a shape is present). */
sg_status eps_grad_vjp_sparse(sg_ctx* ctx, sg_scene* scene, const double* p, int p_on_device,
                              const void* const* e_fwd, const void* const* e_adj, double omega,
                              double* grad, int grad_on_device, void* stream);

/* Number of (sample, column step) pairs whose E_fwd and E_adj values the
 * scene's last eps_grad_vjp_sparse call read (16 bytes each); waits for the
 * device. */
sg_status sg_scene_sparse_reads(sg_scene* scene, int64_t* pairs);

/* Reverse mode with an upstream dF/deps (the chain rule of Sec. "Automatic
 * differentiation based acceleration" through the eps map alone, for callers
 * whose objective reaches eps by other means than eq:1's field product, e.g.
 * an autograd graph): grad_eps is C FP32 planes stored contiguously
 * ([C][Nz][Ny][Nx]); grad_k = sum grad_eps * d eps / d p_k.  With grad_eps =
 * 2 omega Im(E Eadj) it equals eps_grad_vjp up to rounding. */
sg_status eps_grad_vjp_geps(sg_ctx* ctx, sg_scene* scene, const double* p, int p_on_device,
                            const float* grad_eps, double* grad, int grad_on_device, void* stream);

/* Finite-difference baseline (Sec. "Background", Sec. "Automatic differentiation
 * based acceleration"): for every k, re-rasterize the whole grid at p +- h e_k
 * (SG_FD_CENTRAL, 2n rasterizations) or at p + h e_k against p (SG_FD_FORWARD,
 * the paper's n + 1 form), write the difference plane (FP64 difference, stored
 * FP32), then reduce sum_j g_j * diff_j / (2h or h) with g = 2*omega*Im(E Eadj).
 * h in um (> 0).  Uses 2 C-plane FP32 work buffers owned by the scene. */
sg_status eps_grad_fd(sg_ctx* ctx, sg_scene* scene, const double* p, int p_on_device,
                      const void* const* e_fwd, const void* const* e_adj, double omega,
                      double h, int scheme, double* grad, int grad_on_device, void* stream);

/* Finite-difference baseline restricted to where each parameter acts (Sec.
 * "Single-polarization blazed grating coupler in 2D", item (iv); the tracked
 * finite differences of Sec. "Discussion and Conclusion"): same arguments and
 * result as eps_grad_fd up to the order of the sums, but for each k only the
 * in-plane tiles that the support boxes of the primitives referencing p_k
 * meet (at p + h e_k or the other point), and only the column steps where a
 * class is nonzero, are re-rasterized; the difference is multiplied by
 * g = 2*omega*Im(E Eadj) in the same pass (no difference plane).  Parameters
 * that an extrusion bound references re-rasterize every tile.  Uses one
 * C-plane FP32 work buffer owned by the scene. */
sg_status eps_grad_fd_sparse(sg_ctx* ctx, sg_scene* scene, const double* p, int p_on_device,
                             const void* const* e_fwd, const void* const* e_adj, double omega,
                             double h, int scheme, double* grad, int grad_on_device, void* stream);

/* Synthetic fields: n complex64 values each of E_fwd and E_adj (device), from
 * Philox4x32-10 (Salmon et al., SC'11) with counter (i mod 2^32, i div 2^32, 0, 0)
 * and key (seed mod 2^32, seed div 2^32); u_k = (x_k + 1/2) 2^-32 and two
 * Box-Muller pairs: E = sqrt(-2 ln u0) e^{2 pi i u1}, E_adj = sqrt(-2 ln u2) e^{2 pi i u3}
 * (FP32).  Used by the serving loop for requests that carry a field seed. */
sg_status sg_fieldgen(void* e_fwd, void* e_adj, int64_t n, uint64_t seed, void* stream);

/* ---------------------------------------------------------------------------
 * Serving: a continuous-batching loop for gradient requests from many
 * concurrent optimizations (sessions) with different scenes, grid sizes and
 * parameter counts.  A scheduler thread admits queued requests in arrival
 * order while request slots and the HBM budget allow, gives each admitted
 * request its own device buffers (seeded fields, staging, gradient; reused per
 * session; a session with a request in flight takes another buffer only from
 * unused budget, else its next request waits for one of its own, while only a
 * session with nothing in flight frees other sessions' idle buffers), groups admitted requests into batched launches (one kernel launch
 * covers the tiles of every request of the same kernel specialization) and
 * issues batches on several streams in turn, so requests that arrive while
 * others run are admitted and overlap with them on the device.  Completion is
 * tracked with events; results wait in host memory until polled.
 * Each request computes eps_grad_vjp of its session's scene at its own p, with
 * fields drawn by sg_fieldgen from its seed.
 * ------------------------------------------------------------------------- */
typedef struct sg_server sg_server;
typedef struct sg_server_opts {
    int64_t hbm_budget_bytes;   /* device bytes the server's request buffers may hold at once
                                   (> 0), busy or kept idle for a session's next request; 0: the
                                   environment variable SG_HBM_BUDGET (bytes, optional K / M / G
                                   suffix for 2^10 / 2^20 / 2^30), else 8 GiB */
    int32_t max_slots;          /* requests admitted at once (>= 1) */
    int32_t max_batch;          /* requests per batch (>= 1) */
    int32_t n_streams;          /* batches in flight at once, one per stream (1..8) */
    int32_t fake_executor;      /* 1: no device work (scheduling tests); the result of a
                                   request is grad_k = 2 p_k + (seed mod 1000); a batch takes
                                   fake_us plus its estimated time (request_bytes at 4.5 TB/s) */
    int64_t fake_us;
    int64_t max_launch_us;      /* > 0: a batch takes work only up to this many estimated
                                   microseconds (HBM bytes at 4.5 TB/s: 16 per field sample
                                   generated and 16 per sample of the column stream); larger
                                   requests are sliced over several batches of one stream, so
                                   requests that arrive meanwhile do not wait for all of them.
                                   0: every batch takes its requests whole */
} sg_server_opts;
typedef struct sg_req_stats {
    int64_t submit_ns, admit_ns, launch_ns, done_ns;   /* steady-clock times */
    int32_t batch_size;                                /* requests in its batch */
    int32_t pad;
} sg_req_stats;

/* ctx may be NULL only with fake_executor = 1. */
sg_status sg_server_create(sg_ctx* ctx, const sg_server_opts* opts, sg_server** out);
/* Cancels queued requests, waits for launched ones, frees everything. */
sg_status sg_server_destroy(sg_server* server);
/* A session runs its requests on `scene` (which must outlive the server),
 * with the scene's deterministic setting at this call: its gradients are then
 * bitwise the same whether a request runs alone or batched with others. */
sg_status serve_open_session(sg_server* server, sg_scene* scene, uint32_t* session);
/* Fake-executor sessions (scheduling tests): n_params and bytes per request given directly. */
sg_status serve_open_fake_session(sg_server* server, int64_t n_params, int64_t request_bytes, uint32_t* session);
/* Queues a request (p: n_params FP64 on the host, copied).  Never blocks.
 * SG_E_TOO_LARGE if the request can never fit the budget. */
sg_status serve_submit(sg_server* server, uint32_t session, const double* p, uint64_t field_seed, double omega,
                       uint64_t* ticket);
/* Queues a request on the caller's field planes (Sec. "Background": E and
 * E_adj are the solver's outputs, given to step 5): e_fwd, e_adj are arrays
 * of C device pointers to complex64 planes as for eps_grad_vjp.  The pointer
 * arrays are copied; the planes are read by the device work of the request,
 * so they must stay allocated and unchanged until serve_poll has returned
 * the ticket's outcome (or the server is destroyed).  The request holds only
 * staging memory from the budget. */
sg_status serve_submit_fields(sg_server* server, uint32_t session, const double* p, const void* const* e_fwd,
                              const void* const* e_adj, double omega, uint64_t* ticket);
/* Waits up to timeout_us (0: no wait, < 0: forever) for a request.  SG_OK: done,
 * the gradient (n_params FP64) is copied to grad_out (host) and the ticket is
 * retired; SG_EAGAIN: not done yet; SG_E_CANCELLED / SG_E_DEVICE: retired with
 * that outcome.  stats may be NULL. */
sg_status serve_poll(sg_server* server, uint64_t ticket, double* grad_out, int64_t timeout_us, sg_req_stats* stats);
/* Cancels a request: queued requests never run; launched ones finish but their result is dropped. */
sg_status serve_cancel(sg_server* server, uint64_t ticket);
/* Counters: requests completed, batches launched, largest batch, bytes of the
 * requests admitted and not finished, and bytes of every request buffer the
 * server holds (busy, or idle and kept for its session; at most the budget).
 * Any pointer may be NULL. */
sg_status serve_counters(sg_server* server, int64_t* completed, int64_t* batches, int64_t* max_batch_seen,
                         int64_t* bytes_in_use, int64_t* bytes_held);

/* Kernel tracing.  With timing enabled the scene attaches a pair of HIP
 * events to launches of its column kernel (the kernel that evaluates eps or
 * its reverse mode; a call also runs a small staging kernel before it): they
 * take the kernel's own start and end times, dispatch gaps excluded.
 * sg_scene_set_timing(scene, k) with k >= 1 clears the records and then
 * times the 1st, (k+1)-th, (2k+1)-th ... launch of each kind; 0 disables.  sg_scene_kernel_time() waits for the recorded launches
 * of one kind (mode: 0 eps_build, 1 eps_grad_vjp, 2 eps_grad_vjp_geps,
 * 3 eps_grad_fd rasterization, 4 eps_grad_vjp_sparse, 5 eps_grad_fd_sparse) and returns their summed duration (ms) and
 * count. */
sg_status sg_scene_set_timing(sg_scene* scene, int enable);
sg_status sg_scene_kernel_time(sg_scene* scene, int mode, double* total_ms, int64_t* launches);

/* Plain device-to-device copy (bytes a multiple of 16) on `stream`; a
 * reference kernel of known traffic for calibrating HBM byte counters. */
sg_status sg_util_copy(void* dst, const void* src, int64_t bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* SHAPEGRAD_H */

/*
 * kifmm_mi355x.h -- C ABI of the MI355X kernel-independent FMM evaluate for the
 * 3D Laplace kernel K(x, y) = 1 / |x - y| (eq. (2), Section 1).
 *
 * The library computes, for N points that are both sources and targets
 * (Section 2.3), the potentials f(x_i) = sum_j K(x_i, x_j) s_j of eq. (1) and
 * their gradients, approximated by the shared-memory FMM of Algorithm 1
 * (Section 2.1) on a uniform octree: S2U/P2M, U2U/M2M, VLI/M2L, D2D/L2L,
 * D2T/L2P and ULI/P2P, with the operators of Table 1.  Pairs at zero distance
 * contribute nothing.
 *
 * Three objects, each created once and reused (Section 3 notes that a set-up
 * tree serves new source data):
 *   kifmm_tree  -- uniform Morton-ordered octree over the points (host build).
 *   kifmm_ops   -- FP64 operator precompute for an expansion order p.
 *   kifmm_plan  -- tree + operators resident on one GPU, with all device
 *                  workspace allocated; evaluate() runs the FMM on a stream.
 *
 * Conventions for every entry point:
 *   - Return value is a kifmm_status; KIFMM_OK is 0, errors are negative.  No
 *     entry point aborts or lets a C++ exception escape.  On error a message
 *     is available from kifmm_last_error() (thread-local, valid until the
 *     thread's next call into the library).
 *   - Arguments, handles and plan capabilities are validated on the host
 *     before any device work is enqueued or any memory allocated: such errors
 *     (KIFMM_E_INVALID, KIFMM_E_STATE, and KIFMM_E_NOMEM from the device
 *     memory limit) leave nothing enqueued.  A failure reported by the HIP
 *     runtime during an enqueue (KIFMM_E_DEVICE) can leave the kernels
 *     enqueued before it in place; the plan's own streams are joined back into
 *     the caller's stream first, so nothing of the call runs unordered.
 *   - Handles are opaque identifiers, never reused.  A handle that was
 *     destroyed, or was never returned by this library, gives KIFMM_E_STATE
 *     (a null handle: KIFMM_E_INVALID).
 *   - "host" pointers are CPU memory, "device" pointers are HIP device memory
 *     on the plan's device.  The caller owns every pointer it passes; the
 *     library never frees or retains caller memory beyond the call (for
 *     kifmm_evaluate: beyond the point where the stream reaches its last
 *     kernel).
 *   - Streams are hipStream_t values passed as void*; NULL is the null stream
 *     of the current device.
 *   - All per-point arrays are in the caller's input order.
 *   - Objects are not thread-safe; distinct plans may run concurrently on
 *     distinct streams.  A plan holds references to its tree and operators, so
 *     they may be destroyed in any order.
 */
#ifndef KIFMM_MI355X_H
#define KIFMM_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KIFMM_ABI_VERSION 3
#define KIFMM_MAX_DEPTH 10

typedef enum {
  KIFMM_OK = 0,
  KIFMM_E_INVALID = -1, /* an argument is out of range, null or non-finite */
  KIFMM_E_NOMEM = -2,   /* a host or device allocation failed, or would exceed the device memory limit */
  KIFMM_E_DEVICE = -3,  /* the HIP runtime reported an error */
  KIFMM_E_NUMERIC = -4, /* the operator precompute produced a non-finite value */
  KIFMM_E_STATE = -5    /* a destroyed or unknown handle, or a plan created without the capability the call needs */
} kifmm_status;

typedef struct kifmm_tree_s* kifmm_tree;
typedef struct kifmm_ops_s* kifmm_ops;
typedef struct kifmm_plan_s* kifmm_plan;

/* ABI version of the loaded library (KIFMM_ABI_VERSION it was built with). */
int kifmm_abi_version(void);

/* Message of the last failed call on this thread; valid until the next call. */
const char* kifmm_last_error(void);

/* ---------------------------------------------------------------- tree --- */

typedef struct {
  int64_t n;                  /* points */
  int64_t nonempty_leaves;
  int64_t max_leaf;           /* largest leaf occupancy */
  int64_t nonempty_boxes[16]; /* per level 0..depth; 0 beyond depth */
  double center[3];           /* enclosing cube centre */
  double half_width;          /* enclosing cube half-width R0 */
  int depth;                  /* leaf level L */
} kifmm_tree_stats;

/*
 * Build the uniform octree of Section 2.1: the enclosing cube is split
 * recursively into octants down to level `depth`, and points are ordered by
 * the Morton key of their leaf (three bits per level, Section 2.1), ties kept
 * in input order.
 *
 *   xyz    device, [n][3] float, point coordinates (finite, |x| < 1e30), on
 *          the device of `stream`.  The library copies them to the host on
 *          `stream` and waits for the copy; the build itself runs on the host
 *          and nothing remains enqueued when the call returns.
 *   n      number of points, 1 <= n < 2^31.
 *   depth  leaf level L, 0 <= L <= KIFMM_MAX_DEPTH.
 *   cube   host, {cx, cy, cz, half_width} in double, or NULL.  NULL encloses
 *          the points in a cube centred on the midpoint of their per-axis
 *          range with half-width 0.5 * (max range) * (1 + 1e-6).  Points
 *          outside a given cube are clamped into its boundary leaves.
 *   stream the stream that orders the read of xyz after its producer.
 *   out    receives the tree handle.
 *
 * Leaf grid coordinates are i_d = floor((x_d - (c_d - R0)) / h), h = 2 R0 / 2^L,
 * computed in double precision and clamped to [0, 2^L - 1].  The tree owns a
 * host copy of the points; xyz is not read after the call.
 */
kifmm_status kifmm_tree_build(const float* xyz, int64_t n, int depth, const double* cube, void* stream,
                              kifmm_tree* out);
/* The same from host memory (xyz host, [n][3] float); touches no device. */
kifmm_status kifmm_tree_build_host(const float* xyz, int64_t n, int depth, const double* cube, kifmm_tree* out);
/* Shape of a tree (host).  KIFMM_E_INVALID if out is null. */
kifmm_status kifmm_tree_stats_get(kifmm_tree tree, kifmm_tree_stats* out);
/* host, [n] int64: input index of the point at each sorted position. */
kifmm_status kifmm_tree_get_order(kifmm_tree tree, int64_t* order);
/* host, [n][3] int32: leaf grid coordinates of each point, input order. */
kifmm_status kifmm_tree_get_leaf_coords(kifmm_tree tree, int32_t* ijk);
/* Releases the caller's handle (the tree lives on while a plan holds it). */
kifmm_status kifmm_tree_destroy(kifmm_tree tree);

/* ----------------------------------------------------------- operators --- */

typedef struct {
  int32_t p;            /* expansion order */
  int32_t n_surface;    /* 6 (p - 1)^2 + 2 points per check/equivalent surface (Section 4) */
  int32_t rank_m2l;     /* k, rank of the compressed U2D (M2L) operators */
  int32_t rank_c2e;     /* kept singular values of the check-to-equivalent pseudo-inverse */
  int32_t n_m2l_offsets;/* 316 distinct V-list offsets */
  double eps_pinv;
  double eps_svd;       /* as passed (negative: the rank was given) */
  double alpha_inner;   /* upward-equivalent and downward-check surface radius factor */
  double alpha_outer;   /* upward-check and downward-equivalent surface radius factor */
} kifmm_ops_info;

/*
 * Precompute, in FP64 on the host, the Table 1 operators for expansion order
 * p on a box of unit half-width (all are scale-free for the Laplace kernel
 * except the leaf S2U factor, scaled at evaluate time):
 *   - the surface S_p: grid points of {-1, .., 1}^3 with p per edge on the
 *     cube boundary, n = 6 (p - 1)^2 + 2 of them (Section 4);
 *   - the equivalent and check surfaces c + alpha r S_p of a box of centre c
 *     and half-width r: upward equivalent and downward check at alpha_inner,
 *     upward check and downward equivalent at alpha_outer;
 *   - check-to-equivalent pseudo-inverses by truncated SVD (relative cutoff
 *     eps_pinv, never splitting a cluster of equal singular values), kept as
 *     two factors for S2U;
 *   - U2U (M2M) and D2D (L2L) operators for the 8 child positions, each a
 *     product formed in FP64 and rounded once;
 *   - the U2D (M2L) operators of the 316 V-list offsets compressed with a
 *     shared basis (the "BLAS M2L" that exploits the translational symmetry
 *     of Section 2.2): K_t ~ U_k C_t V_k^T.
 *
 *   p            2 <= p <= 12.
 *   alpha_inner  1 < alpha_inner < alpha_outer, alpha_inner + alpha_outer <= 4
 *   alpha_outer  (a V-list source's equivalent surface and the target's check
 *                surface then stay apart: the centres of V-list boxes are at
 *                least 4 r apart in the max norm).  1.05 and 2.95 are the
 *                values every workload here uses.
 *   eps_pinv     in (0, 1): relative pseudo-inverse cutoff (1e-7 suits FP32 use).
 *   eps_svd      in (0, 1): relative M2L compression cutoff, k extended to the
 *                end of a singular-value cluster; or a negative integer -k
 *                (1 <= k <= n) to give the rank directly (also extended to the
 *                end of a cluster).
 *   out          receives the handle.
 */
kifmm_status kifmm_ops_precompute(int p, double alpha_inner, double alpha_outer, double eps_pinv, double eps_svd,
                                  kifmm_ops* out);
kifmm_status kifmm_ops_get_info(kifmm_ops ops, kifmm_ops_info* out);

/* Operator inspection (host FP64 copies, row-major), for tests:
 *   KIFMM_OP_SURFACE     [n][3]            index ignored
 *   KIFMM_OP_UC2E        [n][n]            pinv(K(UC, UE)) at unit half-width
 *   KIFMM_OP_DC2E        [n][n]            pinv(K(DC, DE)) at unit half-width
 *   KIFMM_OP_M2M         [n][n]            child position index 0..7 -> parent
 *   KIFMM_OP_L2L         [n][n]            parent -> child position index 0..7
 *   KIFMM_OP_M2L_U       [n][k]            U_k
 *   KIFMM_OP_M2L_V       [n][k]            V_k
 *   KIFMM_OP_M2L_CORE    [k][k]            C_t for offset index 0..315
 *   KIFMM_OP_M2L_OFFSET  [3] (as doubles)  integer offset t of index 0..315
 *   KIFMM_OP_M2L_POST    [n][k]            DC2E U_k
 * `capacity` is the number of doubles `out` can hold. */
enum {
  KIFMM_OP_SURFACE = 0, KIFMM_OP_UC2E = 1, KIFMM_OP_DC2E = 2, KIFMM_OP_M2M = 3, KIFMM_OP_L2L = 4,
  KIFMM_OP_M2L_U = 5, KIFMM_OP_M2L_V = 6, KIFMM_OP_M2L_CORE = 7, KIFMM_OP_M2L_OFFSET = 8,
  KIFMM_OP_M2L_POST = 9
};
kifmm_status kifmm_ops_get_matrix(kifmm_ops ops, int which, int index, double* out, int64_t capacity);
kifmm_status kifmm_ops_destroy(kifmm_ops ops);

/* ---------------------------------------------------------------- plan --- */

/* Flags of kifmm_plan_create.
 *
 * KIFMM_POTENTIAL / KIFMM_GRADIENT (KIFMM_POT / KIFMM_GRAD): which outputs
 * evaluate may be asked for; at least one.
 *
 * KIFMM_M2L_BF16X3 and KIFMM_M2L_BF16X6 (at most one of them) run the
 * compressed M2L translations (Section 2.2, BLAS M2L) on bfloat16 matrix cores
 * with FP32 accumulation, each operand split into bfloat16 pieces (split
 * bfloat16): two pieces and three products (a0 b0 + a0 b1 + a1 b0, each
 * product to about 3 * 2^-16 relative), or three pieces and six products (to
 * about 2^-24, the accuracy of the plain FP32 path).  KIFMM_M2L_BF16X3 uses
 * the three products at the leaf level and six above it, where the
 * translations carry the far field of more sources.  Everything else stays
 * FP32 and the operators are still computed in FP64.
 *
 * By default the U-list sum (ULI), which does not depend on the far field
 * (Section 2.2), runs on a stream owned by the plan, forked from and joined
 * back into the caller's stream with events, so that it overlaps the upward
 * pass and M2L; KIFMM_SERIAL keeps every kernel on the caller's stream (with
 * the near and far leaf sums fused in one kernel).
 *
 * KIFMM_VJP: allocate the workspace of kifmm_evaluate_vjp (two [n][3] float
 * fields on the device).
 *
 * The plain FP32 M2L of a one-RHS plan has two forms: blocked (targets of a
 * 4 x 4 x 4 block of parents with their sources staged in LDS; best for dense
 * trees) and gathered (32 targets of one level and sibling position per wave,
 * each gathering its own sources; best for sparse trees).  By default
 * kifmm_plan_create times both on the plan's own tables and keeps the faster
 * (stats[7] reports the choice); KIFMM_M2L_BLOCKED / KIFMM_M2L_GATHER force one.
 *
 * A one-RHS plan that is not KIFMM_SERIAL and has depth >= 3 can run the
 * levels above the leaves (U2U, their compression and VLI) on a second plan
 * stream beside the leaf level's VLI.  By default kifmm_plan_create times
 * evaluates both ways and keeps the faster (stats[9]); KIFMM_UPPER_STREAM
 * forces the second stream, KIFMM_NO_UPPER_STREAM forbids it (at most one of
 * the two; either is ignored where the second stream does not apply).
 *
 * Leaf kernels of one-RHS plans (U-list sum and D2T) run 256 or 320 threads
 * per workgroup.  Where the U-list sum has a stream of its own the same
 * timing chooses between them (stats[11]); KIFMM_LEAF_THREADS_256 /
 * KIFMM_LEAF_THREADS_320 force one (at most one of the two).  No result bit
 * depends on the choice.
 *
 * KIFMM_LEAF_QUEUE: one-RHS plans run the U-list sum and D2T as one persistent
 * kernel over a work queue of target tiles (at most 64 targets of one leaf
 * each) instead of one workgroup per parent; for trees with uneven leaves.
 * By default plan creation times both (stats[12]), the queue with 2, 4 and 8
 * workgroups per CU (stats[24]); with KIFMM_LEAF_BLOCKS the per-parent kernel
 * is forced (at most one of the two).
 *
 * Plan creation also times the LDS slab of the blocked FP32 M2L (stats[10],
 * stats[25..28]).  Every timed choice is kept for the process: a later plan of
 * the same shape (device, sizes, order, rank, flags, box and leaf occupancy)
 * takes it without timing (stats[23]).  The leaf kernels' workgroup size and
 * the second stream change no result bit; the M2L form, the LDS slab (the
 * grouping of the FP32 sums over k) and the leaf kernel (blocks or queue)
 * change results at the level of FP32 rounding.  KIFMM_NO_AUTOTUNE times
 * nothing and takes the default of every choice no flag forces: blocked M2L
 * with the slab that keeps the most waves resident, the second stream where it
 * applies, per-parent leaf kernels of 320 threads.
 */
#define KIFMM_POTENTIAL 1u
#define KIFMM_GRADIENT 2u
#define KIFMM_POT KIFMM_POTENTIAL
#define KIFMM_GRAD KIFMM_GRADIENT
#define KIFMM_M2L_BF16X3 4u
#define KIFMM_SERIAL 8u
#define KIFMM_M2L_BF16X6 16u
#define KIFMM_VJP 32u
#define KIFMM_M2L_BLOCKED 64u
#define KIFMM_M2L_GATHER 128u
#define KIFMM_UPPER_STREAM 256u
#define KIFMM_NO_UPPER_STREAM 512u
#define KIFMM_LEAF_THREADS_256 1024u
#define KIFMM_LEAF_THREADS_320 2048u
#define KIFMM_LEAF_QUEUE 4096u
#define KIFMM_LEAF_BLOCKS 8192u
#define KIFMM_NO_AUTOTUNE 16384u

/*
 * Place a tree and its operators on the device of `stream` (the current
 * device for NULL): uploads the sorted points, interaction tables and FP32
 * operators on `stream` and allocates all workspace, so that kifmm_evaluate
 * allocates nothing and never synchronises the host.  Choices left open by
 * the flags are timed on `stream` with evaluates of zero charges.  Blocks
 * until the stream has finished the uploads and the timing.
 *
 * nrhs: right-hand sides per evaluate (charge vectors sharing the points), 1,
 * 2, 4, 8, 16 or 32.  With nrhs > 1 the translations of all right-hand sides
 * run as one batch and the leaf kernels compute each pair's geometry once for
 * all of them; such plans give potentials only (no KIFMM_GRADIENT, no
 * KIFMM_VJP) and run on the caller's stream alone.
 *
 * A tree of depth >= 2 (one with a far field) needs p <= 8 (at most 304
 * surface points, which the leaf kernels hold in LDS); larger p gives
 * KIFMM_E_INVALID.  Depth 0 and 1 (the direct sum) take any p.
 *
 * Device memory: the plan needs the number of bytes kifmm_plan_workspace_bytes
 * reports (its resident arrays plus the buffers of the plan-time timing,
 * which are freed before the call returns).  Above the process-wide limit of
 * kifmm_set_device_memory_limit the call fails with KIFMM_E_NOMEM before any
 * device allocation or enqueue.
 */
kifmm_status kifmm_plan_create(kifmm_tree tree, kifmm_ops ops, int nrhs, unsigned flags, void* stream,
                               kifmm_plan* out);

/* Device bytes kifmm_plan_create would need for these arguments (host work
 * only: no device is touched).  Same argument checks as kifmm_plan_create. */
kifmm_status kifmm_plan_workspace_bytes(kifmm_tree tree, kifmm_ops ops, int nrhs, unsigned flags, int64_t* bytes);

/* Process-wide cap on the device bytes one kifmm_plan_create may allocate;
 * 0 (the initial value) means no cap.  KIFMM_E_INVALID for a negative value. */
kifmm_status kifmm_set_device_memory_limit(int64_t bytes);

/*
 * One FMM evaluate (Algorithm 1) on `stream`, asynchronous with respect to the
 * host.  `stream` must belong to the plan's device.
 *
 *   charges    device, [n][nrhs] float, densities s in input order (the nrhs
 *              right-hand sides of a point contiguous).
 *   potential  device, [n][nrhs] float, receives f in input order; or NULL.
 *   gradient   device, [n][3] float, receives grad f in input order; or NULL
 *              (needs KIFMM_GRADIENT at plan creation, else KIFMM_E_STATE).
 *
 * At least one output must be non-NULL.  The buffers must stay valid until
 * the stream has passed this call's last kernel; the plan may not be used on
 * two streams at once.  Arithmetic is FP32 (operators rounded once from FP64).
 */
kifmm_status kifmm_evaluate(kifmm_plan plan, const float* charges, float* potential, float* gradient,
                            void* stream);

/*
 * Vector-Jacobian product of the evaluate, for a loss L = sum_i w_i f_i with f
 * the potentials of densities s at the points (the differentiation of the
 * evaluate; the plan needs KIFMM_VJP, else KIFMM_E_STATE):
 *
 *   grad_charges[j]   = dL/ds_j = sum_i w_i K(x_i, x_j): the evaluate applied
 *                       to the weights, i.e. the adjoint FMM with sources and
 *                       targets exchanged, which for this symmetric kernel and
 *                       equal source and target sets is the same operator;
 *   grad_points[k][:] = dL/dx_k = w_k grad f_s(x_k) + s_k grad f_w(x_k), the
 *                       field of s weighted by w plus the field of w weighted
 *                       by s (needs KIFMM_GRADIENT).
 *
 *   charges      device, [n] float, s in input order.
 *   weights      device, [n] float, w in input order.
 *   field        device, [n][3] float, grad f_s from an earlier evaluate of the
 *                same charges (saves one evaluate); or NULL, and it is computed.
 *   grad_charges device, [n] float, or NULL.
 *   grad_points  device, [n][3] float, or NULL.
 *
 * At least one output must be non-NULL.  Runs one evaluate of w (and one of s
 * when grad_points is wanted and field is NULL) and an elementwise kernel on
 * `stream`; the same buffer and stream rules as kifmm_evaluate apply.  The
 * tree is fixed: the derivative is that of the evaluate for points that stay
 * in their leaves.
 */
kifmm_status kifmm_evaluate_vjp(kifmm_plan plan, const float* charges, const float* weights, const float* field,
                                float* grad_charges, float* grad_points, void* stream);
/*
 * kifmm_evaluate_vjp without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  The same arguments, results and stream rules as
 * kifmm_evaluate_vjp, but the two [n][3] fields it needs live in a device array
 * of the library (KIFMM_NOALLOC_MAX_POINTS x 6 floats = 48 MiB, held by each
 * GPU the library runs on until the process ends) instead of plan memory, so
 * the plan needs no KIFMM_VJP.  Plans with more than KIFMM_NOALLOC_MAX_POINTS
 * points give KIFMM_E_INVALID, and grad_points needs KIFMM_GRADIENT
 * (KIFMM_E_STATE).  Every call on one GPU shares that array: calls that
 * overlap in time on one GPU (on different streams, or from different threads)
 * race and must be ordered by the caller.  The fields are written in full by
 * each call before they are read, so no call depends on an earlier one's
 * contents.
 */
#define KIFMM_NOALLOC_MAX_POINTS 2097152
kifmm_status kifmm_evaluate_vjp_noalloc(kifmm_plan plan, const float* charges, const float* weights,
                                        const float* field, float* grad_charges, float* grad_points, void* stream);
kifmm_status kifmm_plan_destroy(kifmm_plan plan);

/* ------------------------------------------------- inspection, timing --- */

/* Stages of one evaluate, in launch order. */
enum {
  KIFMM_STAGE_PERMUTE = 0, /* gather charges into sorted order */
  KIFMM_STAGE_P2M = 1,     /* leaf sources -> upward-check field (S2U, first half) */
  KIFMM_STAGE_UC2E = 2,    /* upward-check field -> upward density, two factors */
  KIFMM_STAGE_M2M = 3,     /* U2U, all levels; with the plan's second stream also the compression, VLI
                              and downward pass (post, D2D) of the levels above the leaves and the
                              D2D into the leaf level, which run there beside the leaf VLI */
  KIFMM_STAGE_COMPRESS = 4,/* u -> V_k^T u, levels 2..L (the leaf level alone with the second stream) */
  KIFMM_STAGE_M2L = 5,     /* compressed VLI, all levels (the leaf level alone with the second stream) */
  KIFMM_STAGE_L2L = 6,     /* post (DC2E U_k) and D2D, levels 2..L (with the second stream: the leaf
                              level's post) */
  KIFMM_STAGE_P2P = 7,     /* ULI at the leaves (on the plan's stream), or fused D2T + ULI with KIFMM_SERIAL
                              or the leaf work queue */
  KIFMM_STAGE_L2P = 8,     /* D2T added to the ULI result, written in input order (per-parent leaf
                              kernels on the plan's stream only) */
  KIFMM_N_STAGES = 9
};

/* When enabled, evaluate records HIP events around every stage on its stream
 * and kifmm_plan_get_stage_times returns the summed milliseconds and call counts
 * since the last reset (it synchronises on the recorded events). */
kifmm_status kifmm_plan_set_timing(kifmm_plan plan, int enable);
kifmm_status kifmm_plan_get_stage_times(kifmm_plan plan, double* ms, int64_t* counts, int reset);

/* Plan shape: box counts and work counts used for roofline accounting.
 *   stats[0] = leaf-level pairs (target point, source point) of the U-list sum
 *   stats[1] = V-list (target box, source box) pairs over levels 2..L
 *   stats[2] = leaf slots, stats[3] = M2L target boxes, stats[4] = k, stats[5] = n,
 *   stats[6] = right-hand sides per evaluate,
 *   stats[7] = M2L form: 0 blocked FP32, 1 gathered FP32, 2 wide (32 right-hand sides),
 *              3 split bfloat16,
 *   stats[8] = V-list pairs of the KIFMM_STAGE_M2L launch (the leaf level's
 *              alone when the levels above it run on the plan's second stream),
 *   stats[9] = 1 if the levels above the leaves run on the plan's second stream
 *              beside the leaf level's VLI,
 *   stats[10] = k per LDS slab of the staged M2L sources in the blocked forms
 *              (0 for the other forms),
 *   stats[11] = threads per workgroup of the one-RHS per-parent leaf kernels
 *              (256 or 320); 0 when nrhs > 1,
 *   stats[12] = 1 if the one-RHS leaf sums run as the persistent work-queue
 *              kernel (then stats[13] = its target tiles), else 0,
 *   stats[14..17] = plan-time timing of the evaluate in microseconds (median of
 *              the timed repeats) for [no second stream, 256 threads], [no second
 *              stream, 320], [second stream, 256], [second stream, 320]; 0 where
 *              not timed,
 *   stats[18..19] = plan-time timing of the M2L forms in microseconds
 *              (blocked, gathered); 0 where not timed,
 *   stats[20..21] = plan-time timing of the whole evaluate in microseconds with
 *              the per-parent leaf kernels and with the work queue (each at its
 *              best stream layout); 0 where not timed,
 *   stats[22] = V-list pairs whose target is at the leaf level,
 *   stats[23] = 1 if the timed choices were taken from an earlier plan of the
 *              same shape in this process (nothing was timed),
 *   stats[24] = workgroups per CU of the persistent leaf kernel (0 if unused),
 *   stats[25..28] = plan-time timing of the blocked FP32 M2L (all levels, with
 *              its partial-sum reduction) in microseconds with 24, 32, 40 and 48
 *              k per LDS slab; 0 where not timed.
 * At most `count` entries are written (KIFMM_N_STATS in all).  KIFMM_E_INVALID
 * if stats is null or count is negative. */
#define KIFMM_N_STATS 29
kifmm_status kifmm_plan_get_stats(kifmm_plan plan, int64_t* stats, int count);

/* Copy a level's densities to the host after the stream is idle, as float in
 * the same order as the tree's non-empty boxes at that level (Morton order):
 *   kind 0 = u (upward-equivalent, [boxes][n]), 1 = d (downward-equivalent, [boxes][n]).
 * Synchronises the device. */
kifmm_status kifmm_plan_read_density(kifmm_plan plan, int kind, int level, float* host_out, int64_t capacity);

#ifdef __cplusplus
}
#endif

#endif /* KIFMM_MI355X_H */

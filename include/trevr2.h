/*
 * trevr2.h -- C ABI of an MI355X (gfx950) implementation of TREVR2, the
 * tree-based reverse ray tracer of Wadsley, Baumschlager & Shen (2023,
 * "TREVR2: Illuminating fast N log2 N radiative transfer", MNRAS).
 *
 * Problem solved (Sections 1.2, 2): given gas elements with position, mass
 * m, density rho, per-band opacity kappa_b (per unit mass) and per-band
 * luminosity L_b, return for every *active* element i and band b the
 * element-averaged angle-integrated intensity
 *     J_ib = integral of I_b over solid angle, averaged over the element,
 * (the quantity <4 pi J> of eq. intint; L/(4 pi r^2) far from a lone source
 * in vacuum), computed by tracing N_ray = 12 nside^2 HEALPix beams outward
 * from each bucket of the radiation tree (Sections 2.3-2.6).
 *
 * Conventions for every call:
 *   - Array arguments are DEVICE pointers (hipMalloc'd or torch CUDA tensors)
 *     owned by the caller, unless stated otherwise.  Per-band arrays are
 *     band-major: element (b, i) at [b * n + i].
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Device work is enqueued asynchronously on it; arrays must stay alive
 *     until that work completes.
 *   - The library never allocates device memory: the caller passes the tree
 *     workspace and the scratch buffer, sized with trevr_workspace_bytes.
 *   - Every call returns a trevr_status and never throws.  Parameter and
 *     size errors are found on the host before any launch (TREVR_E_INVALID,
 *     TREVR_E_CAPACITY).  Invalid element data found on the device
 *     (non-positive mass or density, non-finite input) raises a sticky
 *     per-tree flag reported by trevr_check (TREVR_E_DATA).  Per-bucket
 *     buffers that turn out too small during a call (traversal stacks, cut
 *     lists) are handled inside the call, which redoes that step with more
 *     room.  HIP runtime failures map to TREVR_E_HIP with the text in
 *     trevr_last_error().
 */
#ifndef TREVR2_H
#define TREVR2_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TREVR_OK = 0,
  TREVR_E_INVALID = 1,  /* bad parameter, size or NULL pointer            */
  TREVR_E_CAPACITY = 2, /* workspace or scratch too small                  */
  TREVR_E_HIP = 3,      /* HIP runtime error (see trevr_last_error)         */
  TREVR_E_STATE = 4,    /* unknown or destroyed tree handle                 */
  TREVR_E_DATA = 5      /* invalid input data found on the device          */
} trevr_status;

/* Option flags (trevr_params.flags). */
enum {
  TREVR_THICK_CORR = 1u, /* multiply J by (1 - e^-tau)/tau, tau = kappa rho h
                            (Section 2.1, eq. taucorr)                       */
  TREVR_NEAR_FIELD = 2u, /* particle-particle transfer inside the p-p sphere
                            (Section 2.4); off: r_pp = 0                      */
  TREVR_BACKGROUND = 4u, /* isotropic background intensity entering at the
                            root-cube boundary (abstract; Section 4)          */
  TREVR_ABSORPTION_AVG = 8u, /* linear absorption averaging (Section 2.6, the
                            scheme the transmission average replaces): a
                            cell larger than a bucket takes the volume-weighted
                            linear mean of its two halves' absorption
                            coefficients, (a1 + a2)/2 on the split box, halved
                            again for every empty prefix box up to the owned
                            box (vacuum), the same in every direction.  This
                            is the first-order limit of the transmission
                            average; buckets keep sum(kappa m)/sum(m/rho).    */
  TREVR_DIRECTED = 32u,  /* directed rays (Sections 3.4.1, 4; the 'Directed'
                            rows of table escape), for tests with one source
                            at the point trevr_params.target: in every bucket
                            the ray whose pixel holds the direction from the
                            bucket centre to target is aimed exactly at target
                            instead of along its HEALPix centre.  That ray's
                            cell chords, p-p columns, source projections and
                            background exit use the new direction; its
                            transmission averages stay those of its HEALPix
                            direction.  Other rays are unchanged.             */
  TREVR_COMPLEX_SRC = 64u, /* complex source model (Section 2.7, eq. srccomb):
                            the build stores for every node and each of the
                            N_ray directions the length of the ray from its
                            luminosity centre to its box edge and the
                            absorption along it (buckets: their absorption;
                            merged nodes: the children's rays brought to the
                            same projected end, extended through the node
                            with its transmission average or clipped, and
                            combined so that attenuated luminosities add).  A
                            merged source is then attenuated along its own ray
                            toward the receiver and the cell trace stops at
                            that ray's projected end.  Forward only: the
                            adjoint calls return TREVR_E_INVALID.  Tree
                            workspace grows by 8 (1 + B) N_ray bytes per node. */
  TREVR_KEEP_DEPTHS = 16u /* memory for time in the adjoint: the forward keeps
                            each far source's cell optical depth (and each
                            ray's exit depth with TREVR_BACKGROUND) in the
                            scratch, per (bucket, ray group) whose sources fit
                            one window, and compute_J_backward reads them
                            instead of sweeping the cells again.  Off: the
                            adjoint recomputes every ray's optical-depth
                            prefixes from the cut lists.  Results agree to
                            FP32 rounding.  Single trees only (a forest always
                            recomputes).                                      */
};

typedef struct trevr_params {
  int32_t nside;     /* HEALPix N_side, a power of two in [1, 16]; N_ray = 12 nside^2
                        (Sections 1.3, 2.5; paper default 2, i.e. 48 rays)          */
  int32_t leaf_size; /* bucket capacity, >= 1 (Section 2.3; paper default 12)       */
  int32_t n_bands;   /* B in [1, 16] (kernels are compiled per band count; the
                        paper runs up to 10 bands, Section 3.1)                    */
  uint32_t flags;    /* TREVR_* flags                                               */
  double theta;      /* opening parameter theta_rad >= 0 (Section 2.5.2; 0.75)      */
  double rpp_min;    /* lower bound of the p-p radius (>= 0; 0 = paper's rule)      */
  double box[4];     /* root cube {lo_x, lo_y, lo_z, L}; L <= 0: bounding cube of
                        the particles                                              */
  double target[3];  /* with TREVR_DIRECTED: the point the directed ray of each
                        bucket aims at (the source of a single-source test);
                        ignored otherwise                                         */
} trevr_params;

/* Work counters of the last compute_J on a tree (see trevr_get_counters). */
typedef struct trevr_counters {
  int64_t buckets;          /* buckets with >= 1 active element (walked)        */
  int64_t cells;            /* cells used whole: accepted cells + opened buckets */
  int64_t absorber_entries; /* (cell, ray) pairs with a chord beyond r_pp        */
  int64_t source_entries;   /* far sources placed on a ray                       */
  int64_t segments;         /* sum over active i of sum over rays of
                               (1 + absorber entries + source entries)           */
  int64_t near_pairs;       /* sum over active i of its bucket's p-p set size    */
  int64_t max_near;         /* largest p-p set of a bucket                       */
  int64_t nodes;            /* tree nodes                                       */
  int64_t src_pairs;        /* sum over active i of its bucket's far sources     */
  int64_t near_src_triples; /* sum over active i of (luminous p-p elements) x
                               (p-p set size): the p-p source paths tested     */
  int64_t max_cut;          /* longest cut list of a bucket (entries)            */
  int64_t max_stack;        /* deepest traversal stack (entries)                 */
  int64_t near_src_hits;    /* (receiver, luminous p-p element, p-p element)
                               triples whose element absorbs on the path:
                               nearer the source than the receiver and within
                               its size of the segment                        */
  int64_t pp_log_entries;   /* 16-bit entries a forest's p-p job log needs for
                               the element-major p-p source sweep: one per
                               (p-p element, source) job that passes its
                               culling tests, three per wavefront chunk of 64
                               p-p elements with such jobs, one per pass and
                               wavefront (see trevr_forest_job_log)           */
} trevr_counters;

typedef struct trevr_tree trevr_tree; /* opaque host handle */

/*
 * Byte sizes of the two caller-owned device buffers for n elements:
 *   tree_bytes    -- holds the tree (sorted elements, nodes, per-direction
 *                    transmission tables; Sections 2.3, 2.6); must outlive
 *                    the tree handle;
 *   scratch_bytes -- a default size for compute_J scratch (fixed part plus a
 *                    budget of 64 p-p entries per element).  compute_J
 *                    reports TREVR_E_CAPACITY when its p-p lists need more;
 *                    trevr_scratch_needed then gives the exact size.
 * Returns TREVR_E_INVALID for bad parameters or n <= 0.
 */
trevr_status trevr_workspace_bytes(const trevr_params* p, int64_t n, size_t* tree_bytes,
                                   size_t* scratch_bytes);

/*
 * Build the radiation tree (Section 2.3) and its moments (Section 2.6,
 * Fig. sourcecombine): Morton sort, radix-tree topology with buckets of at
 * most leaf_size elements, luminosity sums and centres, bucket absorption
 * sum(kappa m)/sum(m/rho) and per-direction transmission averages.
 *   x, y, z, m, rho : float [n];  kappa, lum : float [n_bands][n] (device).
 *   tree_ws         : device buffer of >= tree_bytes, caller-owned.
 * The inputs are copied (sorted) into tree_ws and may be freed once the
 * stream work completes.  On success *out receives a new handle that borrows
 * tree_ws.  Synchronises `stream` a few times (one per tree level).
 */
trevr_status trevr_build_tree(const trevr_params* p, int64_t n, const float* x, const float* y,
                              const float* z, const float* m, const float* rho,
                              const float* kappa, const float* lum, void* tree_ws,
                              size_t tree_ws_bytes, void* stream, trevr_tree** out);

/*
 * J for the active elements (Sections 2.1-2.6): per active bucket, the p-p
 * radius and set, one tree walk assigning accepted cells to HEALPix rays as
 * absorbers and sources, the ray reduction with projection correction, the
 * p-p near field, the optional background and thick-element correction.
 *   active : uint8 [n] (nonzero = active), NULL = all active.
 *   bg     : float [n_bands] background intensity, used with
 *            TREVR_BACKGROUND; may be NULL otherwise.
 *   J      : double [n_bands][n], input order; rows of inactive elements are
 *            not written.
 *   scratch: device buffer of scratch_bytes bytes.
 * Synchronises `stream` to size the p-p lists and once per batch of 65536
 * buckets after the walks (to see whether a cut list or a traversal stack
 * needs more room).  Returns TREVR_E_CAPACITY, writing no J, if scratch is
 * too small.  Cell optical
 * depths are summed with LDS atomics, so repeated calls agree to FP32
 * rounding of those sums (about 1e-7 relative), not bit for bit.
 */
trevr_status trevr_compute_J(trevr_tree* t, const uint8_t* active, const float* bg, double* J,
                             void* scratch, size_t scratch_bytes, void* stream);

/*
 * trevr_compute_J without a caller scratch buffer, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The scratch comes from a fixed device
 * array of TREVR_NOALLOC_SCRATCH_BYTES inside the library, one per GPU, held
 * from the library's first such call on that GPU until the process ends; the
 * call itself allocates nothing.  Arguments and results as trevr_compute_J
 * (the GPU is the current device, which must be the tree's).  Every call on
 * a GPU shares that GPU's array: calls that overlap on one GPU (several
 * streams or threads) race and must be serialised by the caller; each call
 * clears the part of the array that must start at zero.  A call whose
 * scratch would exceed the array returns TREVR_E_CAPACITY, writing no J
 * (trevr_scratch_needed gives the size it needed).  The cut lists take
 * 16 KiB per bucket of the array, so trees of up to about 2 x 10^4 elements
 * (leaf size 8) fit.
 */
#define TREVR_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
trevr_status trevr_compute_J_noalloc(trevr_tree* t, const uint8_t* active, const float* bg,
                                     double* J, void* stream);

/*
 * Adjoint of trevr_compute_J (reverse-mode derivative; not in the paper,
 * which defines only the forward map of Sections 2.1-2.6).  Given
 * gJ = dE/dJ for a scalar objective E of the J that trevr_compute_J returns
 * with the same active set and bg, writes
 *   gL     : double [n_bands][n]  dE/dL     (input order, every row written)
 *   gkappa : double [n_bands][n]  dE/dkappa
 *   grho   : double [n]           dE/drho   (through h = (m/rho)^(1/3), the
 *                                 bucket absorption, the columns and the
 *                                 thick-element factor)
 * The derivative is that of the piecewise-smooth map with every discrete
 * decision held at its value: tree, opening tests, pixel of each source,
 * p-p sets, the element whose size sets each p-p radius, ray-cell hits.
 * Positions and masses are not differentiated.
 *   gJ     : double [n_bands][n] (device), rows of inactive elements ignored.
 * The forward's bucket setup, walks and p-p columns are needed again.  If
 * the last compute_J (or backward) on this tree used the same scratch
 * buffer, no call on any tree has written that buffer since, and the active
 * set has the same contents (checked on the device with a 64-bit
 * fingerprint of the active indices), they are taken from the scratch as
 * that call left them; otherwise they are recomputed.  The caller must not
 * write the scratch between the calls.  Either
 * way the result is the same.  The rays' optical-depth prefixes are recomputed
 * from the cut lists (with TREVR_KEEP_DEPTHS: read where the forward kept
 * them).  Synchronises `stream` one to three times and needs
 * more scratch than compute_J (accumulators per node, class and band, and a
 * second p-p column buffer, placed after compute_J's part of the scratch):
 * on TREVR_E_CAPACITY trevr_scratch_needed gives the size.
 * Partial sums are formed with atomics (FP32 in LDS, FP64 in device memory),
 * so repeated calls agree to FP32 rounding of those sums, not bit for bit.
 */
trevr_status trevr_compute_J_backward(trevr_tree* t, const uint8_t* active, const float* bg,
                                      const double* gJ, double* gL, double* gkappa,
                                      double* grho, void* scratch, size_t scratch_bytes,
                                      void* stream);

/*
 * Tuning knobs of a tree (support call; results do not depend on them):
 *   TREVR_TUNE_STACK  entries of the small LDS traversal stack, in [64, 1024]
 *                     (default 1024).  A traversal that needs more switches
 *                     the tree to an 8192-entry stack.
 *   TREVR_TUNE_CUT    cut-list entries per bucket tried first, in [64, 2048]
 *                     (default 2048).  A batch with a longer cut list is
 *                     walked again in parts with room for the longest.
 *   TREVR_TUNE_STAGE  words per bucket in which the bucket setup stages its
 *                     p-p set for the list fill, in [0, 4096] (default 4096,
 *                     used rounded down to a multiple of 64).  A set that
 *                     does not fit is found again by a range query (0: every
 *                     set), and its list is in traversal order instead of
 *                     slot order.
 * Returns TREVR_E_INVALID for an unknown key or a value out of range.
 */
enum { TREVR_TUNE_STACK = 0, TREVR_TUNE_CUT = 1, TREVR_TUNE_STAGE = 2 };
trevr_status trevr_tree_tune(trevr_tree* t, int key, int64_t value);

/* Scratch bytes the last compute_J or compute_J_backward on this tree needed
 * (0 before any). */
trevr_status trevr_scratch_needed(const trevr_tree* t, size_t* bytes);

/* Counters of the last compute_J (synchronises the tree's stream). */
trevr_status trevr_get_counters(trevr_tree* t, trevr_counters* host_out);

/* Synchronise the tree's stream and return its sticky device error. */
trevr_status trevr_check(trevr_tree* t);

/* Free the host handle (the workspace stays the caller's). */
trevr_status trevr_tree_destroy(trevr_tree* t);

/* Tree shape: node count, number of stored direction classes, depth and the
 * root cube {lo_x, lo_y, lo_z, L} (host outputs, any may be NULL). */
trevr_status trevr_tree_info(const trevr_tree* t, int64_t* num_nodes, int32_t* num_classes,
                             int32_t* depth, double* root_box);

/*
 * Copy the tree tables to HOST buffers (any may be NULL), nodes in
 * depth-first preorder, child 0 (lower half) first:
 *   perm    int64 [n]        sorted slot -> input index
 *   ints    int64 [nodes][7] first, count, owned prefix length, split bit
 *                            (-1 for buckets), child 0, child 1, next (preorder
 *                            index after the subtree)
 *   box     double [nodes][6] lo xyz, hi xyz
 *   cen     double [nodes][3] luminosity centre (box centre when dark)
 *   Lb      double [nodes][B] luminosity per band;  Lbol double [nodes]
 *   alpha   float [nodes][classes][B] transmission-averaged absorption
 *   ray_class int32 [N_ray]  direction class of each HEALPix ray
 *   kmass   double [nodes]   sum over elements and bands of kappa m
 *   csrc_d  double [nodes][N_ray], csrc_a double [nodes][N_ray][B]: the
 *           complex source model's ray lengths and absorption (only for a
 *           tree built with TREVR_COMPLEX_SRC; TREVR_E_STATE otherwise)
 * Synchronises the tree's stream.
 */
trevr_status trevr_tree_export(trevr_tree* t, int64_t* perm, int64_t* ints, double* box,
                               double* cen, double* Lb, double* Lbol, float* alpha,
                               int32_t* ray_class, double* kmass, double* csrc_d,
                               double* csrc_a);

/*
 * Kernel timing (support call, not part of the method): when enabled, each
 * compute_J records HIP events on its stream around its phases, and
 * trevr_profile_read adds their elapsed times (synchronising the stream):
 *   ms[TREVR_PROF_SETUP]  bucket list, p-p radii and p-p lists
 *   ms[TREVR_PROF_WALK]   tree walks (cut lists)
 *   ms[TREVR_PROF_REDUCE] far-field ray reduction and final J
 *   ms[TREVR_PROF_NEAR]   particle-particle transfer
 *   ms[TREVR_PROF_ADJ_REDUCE] adjoint of the far-field reduction
 *   ms[TREVR_PROF_ADJ_NEAR]   adjoint of the particle-particle transfer
 *   ms[TREVR_PROF_ADJ_TREE]   adjoint of the p-p radii and of the tree
 *                             moments, gradients to input order
 *   ms[TREVR_PROF_PP_SRC]     the p-p source-path kernel alone (part of NEAR)
 *   ms[TREVR_PROF_ADJ_PP_SRC] its adjoint alone (part of ADJ_NEAR)
 * (compute_J_backward also records SETUP, WALK and NEAR for the forward
 * steps it repeats), with launches[] the number of timed launches of each.
 * Totals accumulate from the last enable; `on` = 0 stops recording.
 */
enum { TREVR_PROF_SETUP = 0, TREVR_PROF_WALK = 1, TREVR_PROF_REDUCE = 2, TREVR_PROF_NEAR = 3,
       TREVR_PROF_ADJ_REDUCE = 4, TREVR_PROF_ADJ_NEAR = 5, TREVR_PROF_ADJ_TREE = 6,
       TREVR_PROF_PP_SRC = 7, TREVR_PROF_ADJ_PP_SRC = 8, TREVR_PROF_SLOTS = 9 };
trevr_status trevr_profile_enable(trevr_tree* t, int on);
trevr_status trevr_profile_read(trevr_tree* t, double* ms, int64_t* launches);

/* ------------------------------------------------------------------------
 * Batches of independent scenes (a forest).
 *
 * A simulation with individual time steps (Section 1.2) asks for J of a
 * varying subset of elements in many scenes of very different sizes; the
 * calls below compute them together.  Each scene keeps its own parameters
 * (N_side, band count, theta, bucket size, flags, box, rpp_min) and its own
 * tree; every per-bucket step is one persistent launch over the (scene,
 * bucket) work items of all scenes with the same band count.
 *
 * Concatenated layouts, for scene s with n_s = offsets[s+1] - offsets[s]
 * elements and B_s bands:
 *   x, y, z, m, rho, active, grho : [sum n_s], scene s from offsets[s];
 *   kappa, lum, J, gJ, gL, gkappa : scene s is a [B_s][n_s] band-major block
 *                                   starting at sum_{t<s} B_t n_t;
 *   bg                            : [sum B_s], scene s from sum_{t<s} B_t.
 * Results per scene equal those of trevr_compute_J / _backward on that
 * scene's own tree (trevr_forest_scene) up to FP32 rounding of the sums
 * formed with atomics.
 *
 * Sizes are fixed once by trevr_forest_plan (synchronising).  The p-p radius
 * of a bucket is set by all of its members, active or not, so the plan's
 * all-active bucket setup and walks bound every later call whatever its
 * active set.  After it, trevr_compute_J_batched and
 * trevr_compute_J_backward_batched only enqueue kernels on `stream` -- no
 * synchronisation, allocation or memset -- so they can be captured in a HIP
 * graph and replayed with new active flags, opacities' adjoints etc. in the
 * same buffers.
 * ------------------------------------------------------------------------ */
typedef struct trevr_forest trevr_forest;

/* Workspace bytes of a forest of S scenes: params [S] and offsets [S+1] are
 * HOST arrays, offsets[0] = 0 and every scene non-empty. */
trevr_status trevr_forest_workspace_bytes(const trevr_params* params, int32_t S,
                                          const int64_t* offsets, size_t* ws_bytes);

/* Build the trees of every scene (each as trevr_build_tree, Sections
 * 2.3-2.6) into the caller's workspace ws.  Synchronises `stream`.  The
 * inputs may be freed afterwards; the forest borrows ws. */
trevr_status trevr_build_forest(const trevr_params* params, int32_t S, const int64_t* offsets,
                                const float* x, const float* y, const float* z, const float* m,
                                const float* rho, const float* kappa, const float* lum, void* ws,
                                size_t ws_bytes, void* stream, trevr_forest** out);

/* Plan: bytes of device scratch the planning pass needs, then the pass
 * itself (bucket setup and walks of every scene with all elements active;
 * picks the traversal stack and the cut-list length of every later call).
 * Synchronises `stream`.  Afterwards trevr_forest_scratch_bytes gives the
 * scratch every batched call needs (forward and adjoint alike). */
trevr_status trevr_forest_plan_bytes(const trevr_forest* f, size_t* bytes);
trevr_status trevr_forest_plan(trevr_forest* f, void* scratch, size_t scratch_bytes,
                               void* stream);
trevr_status trevr_forest_scratch_bytes(const trevr_forest* f, size_t* bytes);

/* The p-p job log (memory for time, like TREVR_KEEP_DEPTHS for one tree):
 * with bytes > 0 the batched forward keeps, for its adjoint, the
 * (p-p element, source) jobs of its element-major p-p source sweep (Section
 * 2.4's near-field paths) that passed the culling tests, in up to `bytes`
 * of extra scratch; the adjoint that reuses that forward's state then runs
 * only their exact tests.  The decisions are the forward's own, so results
 * are unchanged (up to the order of FP32 atomic sums).  Buckets whose jobs
 * do not fit, and those the sweep takes pair-major, are culled again by the
 * adjoint.  The counter pp_log_entries (2 bytes each) of a forward gives
 * the size that covers every bucket, plus up to 128 KiB per persistent
 * wavefront and band count for partly used blocks.  0 (the default) turns
 * the log off.  Afterwards trevr_forest_scratch_bytes includes the log; a
 * forward before the change is not reused.  May be called before or after
 * the plan; TREVR_E_STATE for an unknown forest. */
trevr_status trevr_forest_job_log(trevr_forest* f, size_t bytes);

/* J of the active elements of every scene (layouts above; active NULL = all
 * active; bg may be NULL unless a scene has TREVR_BACKGROUND).  Rows of
 * inactive elements are left untouched.  Enqueues kernels only (graph
 * capturable).  TREVR_E_STATE before a plan, TREVR_E_CAPACITY if scratch is
 * smaller than trevr_forest_scratch_bytes. */
trevr_status trevr_compute_J_batched(trevr_forest* f, const uint8_t* active, const float* bg,
                                     double* J, void* scratch, size_t scratch_bytes,
                                     void* stream);

/* Adjoint of trevr_compute_J_batched (same derivative as
 * trevr_compute_J_backward, per scene; every gradient row written).  If the
 * last batched call of this forest was on this scratch and no call has
 * written the scratch since, its bucket setup, walks and p-p columns are
 * used as they are; they must be for the same active set -- checked on the
 * device by fingerprint, a mismatch raising a sticky flag that
 * trevr_forest_check reports as TREVR_E_STATE and filling gL, gkappa and
 * grho with NaN.  Otherwise they are recomputed.  Enqueues kernels only
 * (graph capturable). */
trevr_status trevr_compute_J_backward_batched(trevr_forest* f, const uint8_t* active,
                                              const float* bg, const double* gJ, double* gL,
                                              double* gkappa, double* grho, void* scratch,
                                              size_t scratch_bytes, void* stream);

/*
 * Autotuner of a forest (support call; results do not depend on the choice
 * beyond FP32 rounding of atomic sums).  Candidate launch configurations,
 * numbered 0 .. TREVR_FOREST_CONFIGS - 1 by three bits:
 *   bit 2  bucket order within a band count: heaviest first (0), or scene
 *          by scene with the heaviest first inside each (1);
 *   bit 1  workgroups of each persistent launch: every slot the device can
 *          hold at once (0), or half of them (1);
 *   bit 0  p-p culling boxes of 16 (0) or 8 (1) elements.
 * trevr_forest_autotune runs trevr_compute_J_batched -- and, when gJ is
 * not NULL, trevr_compute_J_backward_batched -- on the given buffers under
 * every candidate (one warm-up run, then `reps` timed runs), keeps the
 * fastest for later calls and writes the mean milliseconds of each to
 * times[TREVR_FOREST_CONFIGS] (host array, may be NULL).  Synchronises.
 * set_config forces a candidate; get_config reads the one in use
 * (0 until tuned).
 */
enum { TREVR_FOREST_CONFIGS = 8 };
trevr_status trevr_forest_autotune(trevr_forest* f, const uint8_t* active, const float* bg,
                                   double* J, const double* gJ, double* gL, double* gkappa,
                                   double* grho, void* scratch, size_t scratch_bytes,
                                   void* stream, int32_t reps, double* times);
trevr_status trevr_forest_set_config(trevr_forest* f, int32_t config);
trevr_status trevr_forest_get_config(const trevr_forest* f, int32_t* config);

/* Kernel timing of the batched calls (support call, as trevr_profile_enable
 * and trevr_profile_read for a tree, same slots; every launch covers all
 * scenes with one band count).  Recording must be off while a call is
 * captured in a HIP graph. */
trevr_status trevr_forest_profile_enable(trevr_forest* f, int on);
trevr_status trevr_forest_profile_read(trevr_forest* f, double* ms, int64_t* launches);

/* Synchronise and report sticky device errors of the forest and its scenes. */
trevr_status trevr_forest_check(trevr_forest* f);
/* Counters of the last batched call: one scene, or scene = -1 for the sum
 * over scenes (maxima for max_near, max_cut, max_stack).  Synchronises. */
trevr_status trevr_forest_get_counters(trevr_forest* f, int32_t scene, trevr_counters* out);
/* The tree of one scene (owned by the forest), for the single-tree calls. */
trevr_status trevr_forest_scene(trevr_forest* f, int32_t scene, trevr_tree** out);
/* Destroy the forest and its scene trees (host handles only). */
trevr_status trevr_forest_destroy(trevr_forest* f);

const char* trevr_status_string(trevr_status s);
/* Text of the last error raised on the calling thread ("" if none). */
const char* trevr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* TREVR2_H */

/*
 * libbbs: batched branch-and-bound 3D scan matching (3D-BBS, Aoki et al.,
 * arXiv 2310.10023) on AMD Instinct MI355X (gfx950).
 *
 * C ABI.  Plain pointers and sizes only.  Every call is synchronous with
 * respect to the host on return (device work is enqueued on the caller's
 * stream, or the library's own, and waited for).  Errors are reported as a
 * negative bbs_status plus a thread-local message from bbs_last_error(); no
 * call aborts or exits the process.
 *
 * Coordinates are metres, angles radians.  Point arrays are row-major n x 3
 * float32 (x, y, z per point).  A pointer flagged *_on_device is a device
 * address readable by the current HIP device (for example a torch tensor's
 * data_ptr()); otherwise it is host memory.  Inputs are borrowed for the
 * duration of the call only.
 */
#ifndef LIBBBS_H
#define LIBBBS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BBS_ABI_VERSION 1
#define BBS_MAX_LEVELS 16

typedef enum {
    BBS_OK = 0,
    BBS_ERR_INVALID_ARG = -1,    /* an argument failed validation; nothing was changed */
    BBS_ERR_OOM = -2,            /* device or host allocation failed */
    BBS_ERR_DEVICE = -3,         /* a HIP runtime call failed */
    BBS_ERR_QUEUE_OVERFLOW = -4, /* the node queue exceeded the workspace capacity */
    BBS_ERR_INTERNAL = -5        /* an internal consistency check failed */
} bbs_status;

/* Opaque multi-resolution voxel map, owned by the library until bbs_free_map. */
typedef struct bbs_map bbs_map;
/* Opaque search workspace (device queue and buffers), owned by the library
 * until bbs_workspace_free.  One workspace serves one bbs_localize call at a
 * time; concurrent calls need one workspace each. */
typedef struct bbs_workspace bbs_workspace;

/* Search ranges per degree of freedom: x, y, z [m], roll, pitch, yaw [rad].
 * Translation leaves are the cells r*i with min <= r*i <= max (Eq. (1)); an
 * angular axis with min == max is fixed at that angle. */
typedef struct {
    float min[6];
    float max[6];
} bbs_search_range;

typedef struct {
    int32_t batch_size;       /* b: pending children are scored once more than b are waiting
                                 (Alg. 2); default 10000 as in Sec. IV */
    int32_t translation_only; /* 1: angular grids at leaf resolution on every level
                                 (Table I "Trans." branching); 0: roto-translational */
    int32_t profile;          /* P >= 1: time every P-th scoring launch with HIP events (fills
                                 score_kernel_ms / score_launches of the result); 0: off */
    int32_t seed_beam;        /* with a prior: width W of the seed beam.  Starting from the W best
                                 initial nodes reaching the threshold, every beam node is
                                 branched, all children scored, and the W best children
                                 reaching the threshold form the next beam, down to the
                                 leaves; "best" is score desc, prior key desc, position asc.
                                 The best beam leaf seeds the incumbent.  Clamped to 64 and
                                 to 2048 / (most children of one node); 0: no beam */
    void *stream;             /* hipStream_t to run on; NULL = the library's own stream */
    const float *prior;       /* NULL, or 1088 host float logits of the proposal network (64
                                 yaw bins, then 32 x 32 translation cells of the search box,
                                 x outer).  The key of a node is the best yaw-bin logit over
                                 the leaf yaws below it plus the best cell logit over the
                                 leaf translations below it (summed in double).  Initial
                                 nodes are scored and queued in descending key (ties:
                                 enumeration order), which orders ties of (score, level); a
                                 non-finite logit disables the prior */
    int32_t persistent;       /* 1: run the search loop as one cooperative persistent kernel
                                 (falls back to per-iteration launches if it cannot launch) */
    int32_t score_items;      /* scoring work items per batch (groups x point splits); sets the
                                 points each wave handles; 0 = default (2048) */
    int32_t graph;            /* 1: capture 8 search iterations in a hipGraph once per search
                                 and replay it (ignored with persistent or profile) */
    int32_t hist_min_level;   /* l >= 1: the pending groups are grouped into runs of one level
                                 and rotation, and runs at level l or above are scored through
                                 the scan's histogram of voxels at that level and rotation
                                 (one lookup per distinct voxel instead of one per point; same
                                 scores); -1: from level 0; 0 (default): off, every group is
                                 scored point by point */
    int32_t strategy;         /* queue order: 0 best first (Alg. 2: score descending, then level
                                 ascending); 1 depth first (the order of Alg. 1, Table I
                                 "DFS": level ascending, then score descending); first in
                                 first out among equal keys, same batching and pruning */
    int32_t rot_exact;        /* 1: exact rotational bound (not in the paper, whose bound is not
                                 strictly exact under rotation, Sec. III-D): nodes of level
                                 l >= 1 are scored against D_l grown by the box margin e_l of
                                 bbs_rotation_margins, so every node bounds every leaf below
                                 it and the result is the full search's optimum (largest
                                 score, lexicographically smallest leaf), whatever the order.
                                 The map must hold grown tables with margins >= e_l
                                 (bbs_build_map_margins), else INVALID_ARG */
    int32_t nested_angles;    /* 1: nested angular cells (not the default reading): Eq. (13) sets
                                 each level's cells on its own, and the children a c + j of
                                 Eq. (14) (a of Eq. (15)) lie inside their parent only when
                                 n_{l-1} = a n_l; otherwise they drift from the parent's angle.
                                 With 1 the grid is built top down: n_lmax as in Eq. (13),
                                 then a_l = ceil((W / n_l) / delta(r_{l-1})) and n_{l-1} =
                                 a_l n_l, so each cell splits into a_l equal children at most
                                 delta(r_{l-1}) wide (a finer leaf grid where the ratios were
                                 not integers).  0 (default): Eq. (13) on every level */
    int32_t reserved3;
} bbs_options;

typedef struct {
    int32_t found;            /* 1: a leaf reached score_threshold; 0: none did */
    int32_t score;            /* hit count of the match, 0..K */
    int32_t leaf[6];          /* leaf index i_x, i_y, i_z, i_roll, i_pitch, i_yaw */
    float pose[6];            /* x = r i_x (cell corner), ..., angles at angular cell centres */
    int64_t nodes_expanded;   /* non-leaf nodes branched */
    int64_t nodes_scored;     /* initial set + every scored child */
    int64_t flushes;          /* scoring batches after the initial set */
    int64_t leaves_accepted;  /* leaf pops with score >= the running best */
    int64_t initial_size;     /* valid nodes at the top level */
    int64_t initial_kept;     /* of those, nodes with score >= score_threshold */
    double score_kernel_ms;   /* duration of the scoring launches (profile >= 1): the sum, or
                                 with profile = P > 1 the mean of the timed ones times their number */
    int64_t score_launches;   /* number of scoring launches (profile >= 1) */
    int64_t score_pairs;      /* sum over scored nodes of K (node-point membership tests) */
    int64_t score_groups;     /* scored groups of translational siblings sharing a rotation */
    double phase_ms[4];       /* set-up, initial set, search loop, total (host clock) */
    int32_t prior_used;       /* 1: the prior ordered the initial set */
    int32_t seeded;           /* 1: the seed beam set the incumbent */
    int32_t seed_score;       /* score of that beam leaf */
    int32_t persistent_used;  /* 1: the search loop ran as one persistent kernel */
    int32_t seed_beam_used;   /* beam width after clamping (0: no beam ran) */
    int32_t reserved_r;
    double serial_ms[4];      /* device time of the serial queue work, summed over iterations
                                 (100 MHz device clock): push, gather, and of push the
                                 bucket prefix over tiles and the chunk allocation */
    int64_t level_groups[BBS_MAX_LEVELS]; /* groups of translational siblings scored per level,
                                 children batches only (0 when every group is scored point
                                 by point, see hist_min_level) */
    int64_t hist_groups;      /* of those, groups scored through a scan histogram */
    int64_t hist_items;       /* histogram work items */
    int32_t hist_fallbacks;   /* histogram items whose scan had too many distinct voxels */
    int32_t hist_off;         /* bit l: level l was switched to point-by-point scoring */
} bbs_result;

/* Fill *opt with the defaults (b = 10000, roto-translational, no profiling,
 * library stream). */
void bbs_default_options(bbs_options *opt);

/* Version of this ABI (BBS_ABI_VERSION). */
int32_t bbs_abi_version(void);

/* Message of the last failed call on this thread ("" if none).  Valid until
 * the next call on this thread. */
const char *bbs_last_error(void);

/*
 * Build the sparse multi-resolution voxel map (Sec. III-C).
 *   xyz, n          map points M (n >= 1), host or device (xyz_on_device)
 *   min_res         r > 0, the level-0 voxel size; level l has voxel 2^l r
 *   levels          l_max in [0, 15]; tables are built for l = 0..l_max
 *   dilate_leaf     1 (default): level 0 is dilated like the coarser levels
 *                   (every occupied voxel v also marks v - j, j in {0,1}^3);
 *                   0: level 0 holds occupied voxels only
 *   stream          hipStream_t or NULL
 *   out             receives the map handle
 * The occupied voxel of a point m at level l is floor(floor(m / r) / 2^l)
 * with the division m / r in float32.  Voxel coordinates must fit in
 * [-2^20, 2^20) (INVALID_ARG otherwise; also for non-finite points).
 */
bbs_status bbs_build_map(const float *xyz, int64_t n, int32_t xyz_on_device, float min_res, int32_t levels,
                         int32_t dilate_leaf, void *stream, bbs_map **out);

/*
 * bbs_build_map, plus the grown tables of the exact rotational bound (option
 * rot_exact): for every level l >= 1 with margins[l] = M > 0, the set D_l
 * grown by the box [-M, M]^3 (every occupied voxel v marks v - j for j in
 * [-M, 1 + M]^3), in the same layout.
 *   margins         NULL (no grown tables) or levels + 1 entries in [0, 8];
 *                   margins[0] is ignored (leaves are scored exactly)
 */
bbs_status bbs_build_map_margins(const float *xyz, int64_t n, int32_t xyz_on_device, float min_res,
                                 int32_t levels, int32_t dilate_leaf, const int32_t *margins, void *stream,
                                 bbs_map **out);

/*
 * The box margins e_l that the exact rotational bound needs (option
 * rot_exact) for scans of largest range d_max searched over `range` on a map
 * of min_res and levels.  A level-l node is scored at the centre rotation of
 * its angular cell; the leaves below it lie within dev_ax of that centre on
 * each axis, so a scan point moves by at most d_max (dev_roll + dev_pitch +
 * dev_yaw), i.e. by D = ceil((that + 1e-5 d_max + 1e-6) / min_res) level-0
 * cells, and e_l = ceil(D / 2^l).  nested_angles as the option of that name.
 * margins: levels + 1 outputs, [0] = 0.
 * A scan of smaller range may need other margins (the angular grid changes
 * with d_max); bbs_localize checks the scan's own.
 */
bbs_status bbs_rotation_margins(float min_res, int32_t levels, double d_max, const bbs_search_range *range,
                                int32_t nested_angles, int32_t *margins);

/*
 * Pose refinement after the search.  The paper takes a BBS pose as good when
 * local registration with GICP can finish from it (Sec. IV, the success
 * criterion; Sec. IV-B aligns the ground truth with GICP) and gives no GICP
 * arithmetic.  Readings: generalized ICP (Segal et al.) with voxel statistics
 * as its distributions.
 *   - Distributions: points grouped by voxel floor(p / voxel) (double); a
 *     voxel of at least min_points points has mean S1 / n and covariance
 *     S2 / n - mu mu^T, regularized plane to plane: eigenvectors U of
 *     ascending eigenvalues, C = U diag(1e-3, 1, 1) U^T.
 *   - The scan's own voxels (same edge, the call's min_points) give each scan
 *     point its covariance C_i; points of smaller scan voxels take no part.
 *   - Pairing: q_i = R p_i + t goes with the nearest target mean among the 27
 *     voxels around floor(q_i / voxel) (lexicographic offsets, the first of
 *     equal distances) if it is closer than one edge.
 *   - Cost: sum of r_i^T Omega_i r_i, r_i = mu - q_i, Omega_i = (C + R C_i
 *     R^T)^-1.  Gauss-Newton on q' = Exp(w) q + tau: J_i = [ [q_i]_x , -I ],
 *     (w, tau) = -(sum J^T Omega J)^-1 sum J^T Omega r, then R <- Exp(w) R,
 *     t <- Exp(w) t + tau; stop after max_iterations steps or once |w| <
 *     eps_rot and |tau| < eps_trans (that step applied).
 */
typedef struct bbs_gicp_target bbs_gicp_target;

/* The target's voxel distributions (device; the points may be freed after
 * the call).  n in [1, 2^30), voxel > 0, min_points >= 4; INVALID_ARG for
 * non-finite points or voxel indices beyond +-2^20. */
bbs_status bbs_gicp_target_create(const float *xyz, int64_t n, int32_t on_device, double voxel, int32_t min_points,
                                  void *stream, bbs_gicp_target **out);
void bbs_gicp_target_free(bbs_gicp_target *target);

typedef struct {
    int32_t max_iterations;   /* Gauss-Newton steps, [0, 1000] (default 20) */
    int32_t min_points;       /* points of a scan voxel that gives a covariance, >= 4 (default 5) */
    double eps_rot;           /* convergence: rotation step below this (rad, default 1e-6) */
    double eps_trans;         /* and translation step below this (m, default 1e-5) */
} bbs_gicp_options;

typedef struct {
    double R[9];              /* refined rotation, row major */
    double t[3];              /* refined translation (m) */
    double cost;              /* cost at the refined pose */
    int64_t pairs;            /* paired scan points at the refined pose */
    int32_t iterations;       /* steps taken */
    int32_t converged;        /* 1: the last step was below both eps */
} bbs_gicp_result;

void bbs_gicp_default_options(bbs_gicp_options *opt);

/* Refine (R0, t0) (sensor to map; R0 row major).  The scan (k x 3 float32,
 * host or device) is prepared on the device per call; the call returns when
 * done.  Allocates its scratch for the duration of the call. */
bbs_status bbs_gicp_refine(const bbs_gicp_target *target, const float *scan, int64_t k, int32_t on_device,
                           const double R0[9], const double t0[3], const bbs_gicp_options *opt, void *stream,
                           bbs_gicp_result *out);

/* One linearization at (R, t): H (6 x 6 row major), g, cost and the number of
 * paired points, in the order (w, tau) of the step. */
bbs_status bbs_gicp_linearize(const bbs_gicp_target *target, const float *scan, int64_t k, int32_t on_device,
                              const double R[9], const double t[3], int32_t min_points, void *stream, double H[36],
                              double g[6], double *cost, int64_t *pairs);

/* Release a map (NULL is ignored). */
void bbs_free_map(bbs_map *map);

/* Lookup layout of level `level` (0..l_max) as the scoring kernel reads it:
 * *dense = 1 if the level's occupancy masks are also held as a dense grid
 * over the brick bounding box (chosen at build time when the grid has at
 * most 4x the hash table's slots), 0 if lookups probe the hash table;
 * *dense_entries = grid entries (16 bytes each), 0 without a grid.  Either
 * output may be NULL.  Membership and scores do not depend on the layout. */
bbs_status bbs_map_layout(const bbs_map *map, int32_t level, int32_t *dense, int64_t *dense_entries);

/* Map facts: l_max, r, and per level the number of voxels in the dilated set
 * D_l, the number of hash slots and of occupied slots.  Arrays of 16. */
bbs_status bbs_map_info(const bbs_map *map, int32_t *levels, float *min_res, int64_t *voxels,
                        int64_t *slots, int64_t *bricks);

/* Copy the voxels of D_level to host memory as (x, y, z) int32 triples, in
 * unspecified order.  *count receives |D_level|; at most cap triples are
 * written. */
bbs_status bbs_map_dump_level(const bbs_map *map, int32_t level, int32_t *out_xyz, int64_t cap,
                              int64_t *count);

/* Membership H^l(v) of n voxels (host int32 triples) in D_level; out[i] is 0
 * or 1 (host). */
bbs_status bbs_map_contains(const bbs_map *map, int32_t level, const int32_t *xyz, int64_t n, uint8_t *out);

/* Workspace for bbs_localize.  max_queue_nodes bounds the node queue (0 =
 * default 64M nodes, 16 B each); the other buffers grow on demand. */
bbs_status bbs_workspace_create(int64_t max_queue_nodes, bbs_workspace **out);
void bbs_workspace_free(bbs_workspace *ws);

/*
 * Global localization of one scan: batched best-first branch and bound
 * (Alg. 2, Sec. III-E) over the roto-translational tree (Sec. III-D), node
 * score = upper bound of Eq. (12).
 *   map, ws         map and workspace (ws NULL: a temporary workspace is used)
 *   scan_xyz, k     scan S (k >= 1), host or device (scan_on_device)
 *   range           search ranges (min <= max per axis, finite)
 *   score_threshold initial best score (Alg. 2); leaves below it are never
 *                   returned.  Above k is allowed and yields found = 0.
 *   opt             options (NULL = defaults)
 *   out             result (caller-allocated)
 * Ties between equal-scoring leaves go to the lexicographically smallest leaf
 * index.  Returns QUEUE_OVERFLOW if the workspace queue fills up.
 */
bbs_status bbs_localize(const bbs_map *map, bbs_workspace *ws, const float *scan_xyz, int64_t k,
                        int32_t scan_on_device, const bbs_search_range *range, int32_t score_threshold,
                        const bbs_options *opt, bbs_result *out);

/* Size of the static device scratch of bbs_localize_noalloc, per GPU. */
#define BBS_NOALLOC_SCRATCH_BYTES (128u << 20)

/*
 * bbs_localize for callers that cannot allocate: serving loops and harnesses
 * that forbid hipMalloc / hipFree (or any allocating library routine) while
 * they run.  The search, arguments and results are those of bbs_localize
 * (without a workspace).  No device memory is allocated or freed and no
 * stream, event or graph is created: every working buffer (scan copies,
 * angle tables, the pending batch, the bucket queue) is carved from one
 * static device array of BBS_NOALLOC_SCRATCH_BYTES per GPU, which the
 * library holds until the process ends.  Host-side set-up still uses small
 * temporary host buffers.
 *   limits          the node queue gets what the other buffers leave (about
 *                   7M nodes for a 10,000-point scan at b = 10,000); a search
 *                   that needs more returns BBS_ERR_QUEUE_OVERFLOW.  A scan
 *                   size / batch size whose other buffers alone do not fit
 *                   returns BBS_ERR_INVALID_ARG.
 *   opt             opt->profile and opt->graph must be 0 (INVALID_ARG
 *                   otherwise); runs on opt->stream, or the null stream if it
 *                   is NULL, and returns when the search is done
 * The scratch keeps whatever the last call left in it; each call clears what
 * must start at zero.  Calls on one GPU share that GPU's scratch, so calls
 * that overlap on one GPU race; calls on different GPUs do not.
 */
bbs_status bbs_localize_noalloc(const bbs_map *map, const float *scan_xyz, int64_t k, int32_t scan_on_device,
                                const bbs_search_range *range, int32_t score_threshold, const bbs_options *opt,
                                bbs_result *out);

/*
 * Score arbitrary nodes with the device scoring kernel (Eq. (12)).
 *   nodes           n host records of 7 int32: level, c_x, c_y, c_z, i_roll,
 *                   i_pitch, i_yaw (angle indices of that level's grid)
 *   scores          n host int32 outputs
 * The angular grid is the one bbs_localize derives from scan and range.
 * Nodes outside the search set are scored all the same (their cell angles
 * are extrapolated from the grid).
 *   mode            bit 0: translation-only grid (as option translation_only);
 *                   bit 1: exact rotational bound (as option rot_exact);
 *                   bit 2: nested angular cells (as option nested_angles)
 */
bbs_status bbs_score_nodes(const bbs_map *map, const float *scan_xyz, int64_t k, const bbs_search_range *range,
                           int32_t mode, const int32_t *nodes, int64_t n, int32_t *scores);

/* One query of a stream. */
typedef struct {
    const float *scan_xyz;    /* k x 3 float32 scan, host or device */
    int64_t k;
    int32_t scan_on_device;
    int32_t score_threshold;
    bbs_search_range range;
    double arrival_s;         /* arrival time in seconds after the start of bbs_serve (>= 0) */
    const float *prior;       /* this query's 1088 proposal logits (host memory, read while the query
                                 runs), or NULL for the prior of the options (if any) */
} bbs_query;

/*
 * Serve a stream of localization queries on one resident map.
 *   queries, n      queries, sorted by arrival_s (not modified)
 *   workers         concurrent searches (1..64); each worker has its own
 *                   workspace and HIP stream, so one query's serial phase
 *                   overlaps the scoring of others; 1 with opt->persistent
 *                   (a persistent search's cooperative grid fills the GPU),
 *                   else BBS_ERR_INVALID_ARG
 *   opt             options for every query (its stream field is ignored; a
 *                   query's own prior, if set, replaces the options' prior)
 *   results         n results, in query order (caller-allocated)
 *   start_s, end_s  n doubles each (caller-allocated, may be NULL): when each
 *                   query started and finished, seconds after the start
 * A query starts at the earliest time at which it has arrived and a worker
 * is free, in arrival order.  The first failing query's status is returned
 * after every worker has finished; its result has found = 0.
 */
bbs_status bbs_serve(const bbs_map *map, const bbs_query *queries, int64_t n, int32_t workers,
                     const bbs_options *opt, bbs_result *results, double *start_s, double *end_s);

/*
 * Learned proposal network (an addition to the paper's method; it orders the
 * initial expansion and seeds the incumbent, never changes a node score).
 * Input: the scan's bird's-eye polar occupancy, 64 range x 64 azimuth bins,
 * uint8 counts.  Output: 1088 float logits, 64 over yaw bins then 32 x 32
 * over translation cells (row-major, x outer).  Weights and activations are
 * bf16 on BF16 MFMA with float accumulation; master weights float.
 * Parameters are one flat float array in the order c1w [16,3,3,1], c1b[16],
 * c2w [32,3,3,16], c2b, c3w [64,3,3,32], c3b, c4w [64,3,3,64], c4b,
 * f1w [256,1024], f1b, f2w [1088,256], f2b (bbs_net_param_count() values).
 */
typedef struct bbs_net bbs_net;

int64_t bbs_net_param_count(void);
/* Network with room for batches of up to max_batch images; parameters zero
 * until bbs_net_set_params. */
bbs_status bbs_net_create(int32_t max_batch, bbs_net **out);
void bbs_net_free(bbs_net *net);
/* Set the float master parameters (host array of count values) and reset the
 * optimiser state. */
bbs_status bbs_net_set_params(bbs_net *net, const float *params, int64_t count);
bbs_status bbs_net_get_params(const bbs_net *net, float *params, int64_t count);
/* Logits of batch images ([batch, 64, 64] uint8, host or device) into a host
 * array of batch x 1088 floats. */
bbs_status bbs_net_forward(bbs_net *net, const uint8_t *images, int32_t images_on_device, int32_t batch,
                           float *logits);
/* One AdamW step (beta 0.9 / 0.999, eps 1e-8, decoupled weight decay on the
 * weights) on the mean cross-entropy of both heads.  yaw[i] in [0, 64),
 * xy[i] in [0, 1024) (host).  lr < 0: compute the gradients only.  loss_out
 * (host float) and grads_out (host, param_count floats) may be NULL. */
bbs_status bbs_net_train_step(bbs_net *net, const uint8_t *images, int32_t images_on_device, const int32_t *yaw,
                              const int32_t *xy, int32_t batch, float lr, float weight_decay, float *loss_out,
                              float *grads_out);
/* The prior of one scan for bbs_localize's opt->prior: the scan's bird's-eye
 * polar image (as bbs_bev_image computes it, d_max included) and the forward
 * pass, on the device, with only the 1088 logits copied to the host array.
 * The scan may be host or device memory; a host scan is staged in a device
 * buffer the network keeps (grown when a larger scan comes).  Runs on the
 * network's own stream and returns when the logits are in place. */
bbs_status bbs_net_prior(bbs_net *net, const float *scan_xyz, int64_t k, int32_t scan_on_device, float *logits);

/* Bird's-eye polar image of a scan into a host [64, 64] uint8 array: range
 * bin floor(64 |(x, y)| / d_max) clamped to 63, azimuth bin
 * floor(64 atan2(y, x) / 2 pi) mod 64, min(255, count) per cell. */
bbs_status bbs_bev_image(const float *scan_xyz, int64_t k, int32_t scan_on_device, uint8_t *image);

/* One measured configuration of bbs_autotune. */
typedef struct {
    int32_t batch_size;
    int32_t score_items;
    double ms;                /* wall time of the sample queries, summed */
} bbs_tune_entry;

/*
 * Pick the node-batch size b and the scoring tile size (points per wave, via
 * score_items) that localize the sample queries fastest: each candidate pair
 * runs every query once after one warm-up query, on one workspace.
 *   batch_sizes, n_b       candidate b values (each in [1, 2^24])
 *   score_items, n_items   candidate score_items values (each in [1, 2^20])
 *   base                   other options (its batch_size and score_items are replaced;
 *                          a query's own prior replaces its prior)
 *   best                   fastest pair (caller-allocated)
 *   all                    NULL or n_b * n_items entries, b outer
 * Note: b changes the search schedule (node counts) but not its rules.
 */
bbs_status bbs_autotune(const bbs_map *map, const bbs_query *queries, int64_t n, const int32_t *batch_sizes,
                        int32_t n_b, const int32_t *score_items, int32_t n_items, const bbs_options *base,
                        bbs_tune_entry *best, bbs_tune_entry *all);

/*
 * Achievable memory rates of the current GPU (measurement only; the search
 * never calls it): the denominators of the scoring kernel's memory roofline.
 * Not from the paper, which reports no kernel rates.
 *   kind 0          streaming read: every 16-byte word of a table_bytes
 *                   buffer read once per pass (several passes), coalesced
 *   kind 1          random gathers: `loads` independent 8-byte loads at
 *                   hashed positions of a table of at most table_bytes (the
 *                   largest power of two of 8-byte entries that fits)
 *   table_bytes     in [4096, 2^36]; loads (kind 1) in [1, 2^34]
 *   gbs, ms         useful bytes per second / 1e9 (kind 1: 8 bytes per load)
 *                   and the kernel time, best of five timed runs (host)
 * Allocates the table for the duration of the call.
 */
bbs_status bbs_bandwidth_probe(int32_t kind, int64_t table_bytes, int64_t loads, double *gbs, double *ms);

/*
 * Scan preprocessing, the step before the search: alignment with the measured
 * gravity direction (Sec. III-A assumes the scan roughly aligned with gravity;
 * Sec. IV-B aligns each scan with the IMU's average acceleration), then the
 * voxel-grid filter that brings scans to about 1,000 points (Sec. IV).
 *   gravity        accelerometer reading in the scan frame (points up when the
 *                  sensor rests); all zero: no alignment.  The scan is rotated
 *                  by the smallest rotation taking g / |g| to +z (yaw is left
 *                  free): with a = g / |g| and k = 1 / (1 + a_z),
 *                  R = [[1 - k a_x a_x, -k a_x a_y, -a_x], [-k a_x a_y,
 *                  1 - k a_y a_y, -a_y], [a_x, a_y, a_z]] formed in double and
 *                  rounded to float (diag(1, -1, -1) when 1 + a_z < 1e-9);
 *                  each coordinate is (R_i0 x + R_i1 y) + R_i2 z in float32
 *   leaf           voxel edge in m, 0 (no filter) or at least 2^-10.  A point's
 *                  voxel is floor(float32(p / leaf)) per axis; each occupied
 *                  voxel becomes the mean of its points, summed exactly as
 *                  integers in units of 2^-24 m (so independent of order) and
 *                  rounded once to float; voxels come out in the order of their
 *                  first point.  Coordinates must be finite and below 1024 m.
 *   target_points  > 0: the leaf is chosen instead, by 24 bisection steps in
 *                  float on [2^-10, max(2 * extent, 1)] m (extent: the largest
 *                  per-axis max - min after alignment): a voxel count above the
 *                  target moves the lower end up, otherwise the upper end
 *                  down; the final upper end is the leaf
 */
typedef struct bbs_preprocess_options {
    float gravity[3];
    float leaf;
    int64_t target_points;
} bbs_preprocess_options;

/*
 * Align and filter one scan (see bbs_preprocess_options).
 *   xyz, n         n x 3 float32 points (x, y, z), n < 2^31; host memory if
 *                  on_device is 0, device memory otherwise
 *   out_xyz        out_cap x 3 float32 points on the same side as xyz
 *                  (caller-allocated; out_cap = n always suffices)
 *   out_n          receives the number of output points; when it exceeds
 *                  out_cap the call writes no points and returns
 *                  BBS_ERR_INVALID_ARG with *out_n set
 *   leaf_used      NULL or receives the leaf of the filter (0: none)
 *   stream         hipStream_t or NULL; the call returns after the stream has
 *                  finished its work
 * Allocates its device scratch (about 40 bytes per point) for the duration of
 * the call.
 */
bbs_status bbs_preprocess_scan(const float *xyz, int64_t n, int32_t on_device, const bbs_preprocess_options *opt,
                               float *out_xyz, int64_t out_cap, int64_t *out_n, float *leaf_used, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* LIBBBS_H */

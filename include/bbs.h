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
    int32_t profile;          /* 1: time every scoring launch with HIP events (fills
                                 score_kernel_ms / score_launches of the result) */
    int32_t reserved0;
    void *stream;             /* hipStream_t to run on; NULL = the library's own stream */
    int64_t reserved[4];
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
    double score_kernel_ms;   /* summed duration of the scoring launches (profile = 1) */
    int64_t score_launches;   /* number of scoring launches (profile = 1) */
    int64_t score_pairs;      /* sum over scored nodes of K (node-point membership tests) */
    int64_t score_groups;     /* scored groups of translational siblings sharing a rotation */
    double phase_ms[4];       /* set-up, initial set, search loop, total (host clock) */
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

/* Release a map (NULL is ignored). */
void bbs_free_map(bbs_map *map);

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
 * score = upper bound of Eq. (eq:3Dupperbound).
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

/*
 * Score arbitrary nodes with the device scoring kernel (Eq. (eq:3Dupperbound)).
 *   nodes           n host records of 7 int32: level, c_x, c_y, c_z, i_roll,
 *                   i_pitch, i_yaw (angle indices of that level's grid)
 *   scores          n host int32 outputs
 * The angular grid is the one bbs_localize derives from scan and range.
 * Nodes outside the search set are scored all the same (their cell angles
 * are extrapolated from the grid).
 */
bbs_status bbs_score_nodes(const bbs_map *map, const float *scan_xyz, int64_t k, const bbs_search_range *range,
                           int32_t translation_only, const int32_t *nodes, int64_t n, int32_t *scores);

#ifdef __cplusplus
}
#endif

#endif /* LIBBBS_H */

/*
 * CPU oracle for 3D-BBS global localization (Aoki et al., "3D-BBS: Global
 * Localization for 3D Point Cloud Scan Matching Using Branch-and-Bound
 * Algorithm", arXiv 2310.10023).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the HIP library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or helper with the HIP library.
 *
 * Every function follows the paper's text in the order it states things:
 *   - multi-resolution voxel map and its dilation ........ Sec. III-C
 *   - node score = upper bound, Eq. (12) .................. Sec. III-C
 *   - rotational step delta(r), Eq. (2) ................... Sec. III-B
 *   - per-level step delta'(r_l) Eq. (13), divisions a Eq. (15) Sec. III-D
 *   - roto-translational branching, Eq. (14) .............. Sec. III-D
 *   - best-first batched search, Alg. 2 ................... Sec. III-E
 * Where the paper is silent the reading used is stated at the point of use.
 *
 * Precision: the rotation entries are formed in double and rounded once to
 * float; the point transform, the division by the voxel size and the floor are
 * float, evaluated in a fixed order (build with -ffp-contract=off, no fast
 * math).  Everything after the floor is integer.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_LEVELS 16
#define ORC_KEY_BIAS (1 << 20)

enum { ORC_OK = 0, ORC_ERR_ARG = -1, ORC_ERR_OOM = -2 };

/* ------------------------------------------------------------------ helpers */

/* floor(v / 2^l) written out, without relying on the shift of a negative int */
static int32_t floor_div_pow2(int32_t v, int l)
{
    int32_t d = (int32_t)1 << l;
    if (v >= 0) return v / d;
    return -((-v + d - 1) / d);
}

static int key_in_range(int32_t x, int32_t y, int32_t z)
{
    return x >= -ORC_KEY_BIAS && x < ORC_KEY_BIAS && y >= -ORC_KEY_BIAS && y < ORC_KEY_BIAS &&
           z >= -ORC_KEY_BIAS && z < ORC_KEY_BIAS;
}

static int64_t pack_key(int32_t x, int32_t y, int32_t z)
{
    return ((int64_t)(x + ORC_KEY_BIAS) << 42) | ((int64_t)(y + ORC_KEY_BIAS) << 21) |
           (int64_t)(z + ORC_KEY_BIAS);
}

static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

static int64_t sort_unique(int64_t *v, int64_t n)
{
    if (n == 0) return 0;
    qsort(v, (size_t)n, sizeof(int64_t), cmp_i64);
    int64_t m = 1;
    for (int64_t i = 1; i < n; ++i)
        if (v[i] != v[m - 1]) v[m++] = v[i];
    return m;
}

/* ------------------------------------------------------------------ map (Sec. III-C) */

typedef struct {
    float r;                           /* minimum voxel size r */
    int32_t levels;                    /* l_max: tables exist for l = 0..l_max */
    int32_t dilate_leaf;               /* 1: level 0 is dilated like every other level */
    int64_t n_keys[ORC_MAX_LEVELS];
    int64_t *keys[ORC_MAX_LEVELS];     /* sorted set D_l of packed voxel keys */
    int32_t margin[ORC_MAX_LEVELS];    /* M_l > 0: keys_rot[l] exists (l >= 1) */
    int64_t n_rot[ORC_MAX_LEVELS];
    int64_t *keys_rot[ORC_MAX_LEVELS]; /* D_l grown by the box [-M_l, M_l]^3 (exact rotational bound) */
} orc_map;

void orc_free_map(orc_map *m)
{
    if (!m) return;
    for (int l = 0; l < ORC_MAX_LEVELS; ++l) {
        free(m->keys[l]);
        free(m->keys_rot[l]);
    }
    free(m);
}

/*
 * Build D_l for l = 0..levels.
 * Occupied voxels at level l are v = floor(p / r_l) with r_l = 2^l r (Sec. III-C).
 * Reading: v is computed as floor(float(p / r)) at level 0 and then divided by
 * 2^l with floor division, which equals floor(p / r_l) in exact arithmetic and
 * keeps the levels nested.
 * Dilation: every occupied voxel also contributes its neighbours v - j for
 * j in {0,1}^3 (V_add, Sec. III-C), at every level (level 0 too unless
 * dilate_leaf is 0).
 */
/*
 * With margins (NULL, or levels + 1 entries of which [0] is unused), every
 * level l >= 1 with M_l = margins[l] > 0 also gets D_l grown by the box
 * [-M_l, M_l]^3, i.e. every occupied voxel contributes v - j for j in
 * [-M_l, 1 + M_l]^3.  These are the tables of the exact rotational bound (see
 * orc_rotation_margins).
 */
int orc_build_map_margins(const float *xyz, int64_t n, float r, int32_t levels, int32_t dilate_leaf,
                          const int32_t *margins, orc_map **out)
{
    *out = NULL;
    if (!xyz || n < 1 || !(r > 0.0f) || !isfinite(r) || levels < 0 || levels >= ORC_MAX_LEVELS)
        return ORC_ERR_ARG;
    int32_t rot_margin = 0;    /* the largest margin, for the scratch size */
    if (margins)
        for (int l = 1; l <= levels; ++l) {
            if (margins[l] < 0 || margins[l] > 8) return ORC_ERR_ARG;
            if (margins[l] > rot_margin) rot_margin = margins[l];
        }
    orc_map *m = (orc_map *)calloc(1, sizeof(orc_map));
    if (!m) return ORC_ERR_OOM;
    m->r = r;
    m->levels = levels;
    m->dilate_leaf = dilate_leaf;
    if (margins)
        for (int l = 1; l <= levels; ++l) m->margin[l] = margins[l];
    /* occupied level-0 voxels, as a set: duplicates change no D_l */
    int64_t *occ = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!occ) { orc_free_map(m); return ORC_ERR_OOM; }
    for (int64_t i = 0; i < n; ++i) {
        int32_t v[3];
        for (int a = 0; a < 3; ++a) {
            float c = xyz[3 * i + a];
            if (!isfinite(c)) { free(occ); orc_free_map(m); return ORC_ERR_ARG; }
            float q = c / r;
            double f = floor((double)q);
            if (f < -(double)ORC_KEY_BIAS + 2 || f >= (double)ORC_KEY_BIAS - 2) {
                free(occ); orc_free_map(m); return ORC_ERR_ARG;
            }
            v[a] = (int32_t)f;
        }
        occ[i] = pack_key(v[0], v[1], v[2]);
    }
    int64_t n_occ = sort_unique(occ, n);
    const int64_t span = 2 + 2 * (int64_t)rot_margin;     /* offsets per axis of the grown tables */
    const int64_t per = span * span * span > 8 ? span * span * span : 8;
    int64_t *buf = (int64_t *)malloc((size_t)n_occ * per * sizeof(int64_t));
    if (!buf) { free(occ); orc_free_map(m); return ORC_ERR_OOM; }
    for (int l = 0; l <= levels; ++l) {
        int dilate = (l > 0) || dilate_leaf;
        int64_t cnt = 0;
        for (int64_t i = 0; i < n_occ; ++i) {
            int32_t vx = floor_div_pow2((int32_t)((occ[i] >> 42) & 0x1FFFFF) - ORC_KEY_BIAS, l);
            int32_t vy = floor_div_pow2((int32_t)((occ[i] >> 21) & 0x1FFFFF) - ORC_KEY_BIAS, l);
            int32_t vz = floor_div_pow2((int32_t)(occ[i] & 0x1FFFFF) - ORC_KEY_BIAS, l);
            if (!dilate) { buf[cnt++] = pack_key(vx, vy, vz); continue; }
            for (int jx = 0; jx <= 1; ++jx)
                for (int jy = 0; jy <= 1; ++jy)
                    for (int jz = 0; jz <= 1; ++jz)
                        buf[cnt++] = pack_key(vx - jx, vy - jy, vz - jz);
        }
        cnt = sort_unique(buf, cnt);
        m->keys[l] = (int64_t *)malloc((size_t)(cnt ? cnt : 1) * sizeof(int64_t));
        if (!m->keys[l]) { free(occ); free(buf); orc_free_map(m); return ORC_ERR_OOM; }
        memcpy(m->keys[l], buf, (size_t)cnt * sizeof(int64_t));
        m->n_keys[l] = cnt;
        if (l > 0 && m->margin[l] > 0) {
            const int32_t M = m->margin[l];
            cnt = 0;
            for (int64_t i = 0; i < n_occ; ++i) {
                int32_t vx = floor_div_pow2((int32_t)((occ[i] >> 42) & 0x1FFFFF) - ORC_KEY_BIAS, l);
                int32_t vy = floor_div_pow2((int32_t)((occ[i] >> 21) & 0x1FFFFF) - ORC_KEY_BIAS, l);
                int32_t vz = floor_div_pow2((int32_t)(occ[i] & 0x1FFFFF) - ORC_KEY_BIAS, l);
                for (int jx = -M; jx <= 1 + M; ++jx)
                    for (int jy = -M; jy <= 1 + M; ++jy)
                        for (int jz = -M; jz <= 1 + M; ++jz)
                            buf[cnt++] = pack_key(vx - jx, vy - jy, vz - jz);
            }
            cnt = sort_unique(buf, cnt);
            m->keys_rot[l] = (int64_t *)malloc((size_t)(cnt ? cnt : 1) * sizeof(int64_t));
            if (!m->keys_rot[l]) { free(occ); free(buf); orc_free_map(m); return ORC_ERR_OOM; }
            memcpy(m->keys_rot[l], buf, (size_t)cnt * sizeof(int64_t));
            m->n_rot[l] = cnt;
        }
    }
    free(occ);
    free(buf);
    *out = m;
    return ORC_OK;
}

int orc_build_map(const float *xyz, int64_t n, float r, int32_t levels, int32_t dilate_leaf, orc_map **out)
{
    return orc_build_map_margins(xyz, n, r, levels, dilate_leaf, NULL, out);
}

int64_t orc_map_level_size(const orc_map *m, int32_t l)
{
    if (!m || l < 0 || l > m->levels) return -1;
    return m->n_keys[l];
}

/* Dump D_l as (x, y, z) triples in increasing packed-key order. */
int64_t orc_map_level_keys(const orc_map *m, int32_t l, int32_t *out_xyz, int64_t cap)
{
    if (!m || l < 0 || l > m->levels) return -1;
    int64_t n = m->n_keys[l] < cap ? m->n_keys[l] : cap;
    for (int64_t i = 0; i < n; ++i) {
        int64_t k = m->keys[l][i];
        out_xyz[3 * i + 0] = (int32_t)((k >> 42) & 0x1FFFFF) - ORC_KEY_BIAS;
        out_xyz[3 * i + 1] = (int32_t)((k >> 21) & 0x1FFFFF) - ORC_KEY_BIAS;
        out_xyz[3 * i + 2] = (int32_t)(k & 0x1FFFFF) - ORC_KEY_BIAS;
    }
    return m->n_keys[l];
}

static int32_t set_contains(const int64_t *k, int64_t n, int32_t x, int32_t y, int32_t z)
{
    if (!key_in_range(x, y, z)) return 0;
    int64_t key = pack_key(x, y, z);
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (k[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo < n && k[lo] == key;
}

/* H^l(v): binary occupancy of voxel v in the dilated level-l map (Sec. III-C). */
int32_t orc_map_contains(const orc_map *m, int32_t l, int32_t x, int32_t y, int32_t z)
{
    return set_contains(m->keys[l], m->n_keys[l], x, y, z);
}

/* The same in the grown table of the exact rotational bound (l >= 1). */
int32_t orc_map_contains_rot(const orc_map *m, int32_t l, int32_t x, int32_t y, int32_t z)
{
    if (l < 1 || !m->keys_rot[l]) return -1;
    return set_contains(m->keys_rot[l], m->n_rot[l], x, y, z);
}

/* ------------------------------------------------------------------ search grid */

typedef struct {
    int32_t levels;
    int32_t translation_only;
    float r;
    double dmax;                           /* largest scan range d_max */
    double delta[ORC_MAX_LEVELS];          /* delta(r_l), Eq. (2) with r -> r_l */
    int32_t n[3][ORC_MAX_LEVELS];          /* angular cells per axis (roll, pitch, yaw) */
    double dprime[3][ORC_MAX_LEVELS];      /* delta'(r_l), Sec. III-D */
    int32_t a[3][ORC_MAX_LEVELS];          /* divisions a from level l to l - 1 (l >= 1) */
    double wmin[3], wmax[3];               /* angular ranges */
    int32_t lo[3], hi[3];                  /* leaf translation index range per axis */
    double tmin[3], tmax[3];               /* translation ranges [m] */
    int32_t rot_exact;                     /* 1: inner nodes are scored against the grown tables */
    int32_t pad;
} orc_grid;

/*
 * Angular and translational discretisation.
 *  delta(r) = arccos(1 - r^2 / (2 d_max^2))                       Eq. (2)
 *  delta'(r_l) = W / ceil(W / delta(r_l)),   W = W_max - W_min      Sec. III-D
 *  a = ceil(delta'(r_l) / delta'(r_{l-1})) if delta'(r_{l-1}) < W else 1.
 * Readings: d_max = largest |s_k| (double); the arccos argument is clamped to
 * [-1, 1]; an axis with W = 0 has one cell; n_l = ceil(W / delta_l) cells of
 * width delta'_l = W / n_l, so delta'_l / delta'_{l-1} = n_{l-1} / n_l and
 * a = ceil(n_{l-1} / n_l) (which is 1 exactly when n_{l-1} = 1).  In
 * translation-only mode (Table I, "Trans.") every level keeps the leaf grid.
 * Translation: leaf indices i with W_min <= r i <= W_max (the set of Eq. (1)),
 * i.e. [ceil(W_min / r), floor(W_max / r)].
 */
int orc_setup(const float *scan, int64_t k, const float rmin[6], const float rmax[6], float r,
              int32_t levels, int32_t translation_only, orc_grid *g)
{
    memset(g, 0, sizeof(*g));
    if (!scan || k < 1 || !(r > 0.0f) || levels < 0 || levels >= ORC_MAX_LEVELS) return ORC_ERR_ARG;
    for (int i = 0; i < 6; ++i)
        if (!isfinite(rmin[i]) || !isfinite(rmax[i]) || rmin[i] > rmax[i]) return ORC_ERR_ARG;
    g->levels = levels;
    g->translation_only = translation_only;
    g->r = r;
    double dmax = 0.0;
    for (int64_t i = 0; i < k; ++i) {
        double x = scan[3 * i], y = scan[3 * i + 1], z = scan[3 * i + 2];
        if (!isfinite(x) || !isfinite(y) || !isfinite(z)) return ORC_ERR_ARG;
        double d = sqrt(x * x + y * y + z * z);
        if (d > dmax) dmax = d;
    }
    g->dmax = dmax;
    for (int l = 0; l <= levels; ++l) {
        double rl = ldexp((double)r, l);
        double c = 1.0 - (rl * rl) / (2.0 * dmax * dmax);
        if (c < -1.0) c = -1.0;
        if (c > 1.0) c = 1.0;
        g->delta[l] = acos(c);
    }
    for (int ax = 0; ax < 3; ++ax) {
        g->wmin[ax] = rmin[3 + ax];
        g->wmax[ax] = rmax[3 + ax];
        double W = g->wmax[ax] - g->wmin[ax];
        for (int l = 0; l <= levels; ++l) {
            int src = translation_only ? 0 : l;
            int32_t n;
            if (W == 0.0) n = 1;
            else {
                double q = ceil(W / g->delta[src]);
                if (!(q >= 1.0)) q = 1.0;
                if (q > 1.0e8) return ORC_ERR_ARG;
                n = (int32_t)q;
            }
            g->n[ax][l] = n;
            g->dprime[ax][l] = W / n;
        }
        g->a[ax][0] = 1;
        for (int l = 1; l <= levels; ++l)
            g->a[ax][l] = (g->n[ax][l - 1] + g->n[ax][l] - 1) / g->n[ax][l];
    }
    for (int ax = 0; ax < 3; ++ax) {
        g->tmin[ax] = rmin[ax];
        g->tmax[ax] = rmax[ax];
        double lo = ceil((double)rmin[ax] / (double)r);
        double hi = floor((double)rmax[ax] / (double)r);
        if (lo > hi) return ORC_ERR_ARG;
        if (lo < -(double)ORC_KEY_BIAS / 4 || hi > (double)ORC_KEY_BIAS / 4) return ORC_ERR_ARG;
        g->lo[ax] = (int32_t)lo;
        g->hi[ax] = (int32_t)hi;
    }
    /* every transformed key must stay inside the packable range */
    if (dmax / r + 4.0 >= (double)ORC_KEY_BIAS / 4) return ORC_ERR_ARG;
    return ORC_OK;
}

/*
 * Nested angular cells (an alternative reading, not the default).  With
 * delta'_l = W / n_l per level (Eq. (13)) and the children a c + j of
 * Eq. (14), a = ceil(n_{l-1} / n_l) (Eq. (15)), a child cell lies inside its
 * parent only when n_{l-1} = a n_l; otherwise children drift away from their
 * parent's angle (with a = 3 where n_{l-1} is just above 2 n_l, level-l cell
 * c has children at about 1.5 times its angle).  This builds the grid top
 * down instead: n_lmax as in Eq. (13), then a_l = ceil((W / n_l) /
 * delta(r_{l-1})) and n_{l-1} = a_l n_l, so every cell splits into a_l equal
 * children, each at most delta(r_{l-1}) wide.  Translation-only grids and
 * axes with W = 0 are unchanged.
 */
int orc_grid_nest(orc_grid *g)
{
    if (g->translation_only) return ORC_OK;
    for (int ax = 0; ax < 3; ++ax) {
        double W = g->wmax[ax] - g->wmin[ax];
        if (W == 0.0) continue;
        for (int l = g->levels; l >= 1; --l) {
            double a = ceil((W / g->n[ax][l]) / g->delta[l - 1]);
            if (!(a >= 1.0)) a = 1.0;
            if (a * g->n[ax][l] > 1.0e8) return ORC_ERR_ARG;
            g->n[ax][l - 1] = (int32_t)(a * g->n[ax][l]);
        }
        for (int l = 0; l <= g->levels; ++l) g->dprime[ax][l] = W / g->n[ax][l];
        g->a[ax][0] = 1;
        for (int l = 1; l <= g->levels; ++l) g->a[ax][l] = g->n[ax][l - 1] / g->n[ax][l];
    }
    return ORC_OK;
}

/* Angle of cell c of axis ax at level l.  Reading: cells are anchored at their
 * centres, W_min + delta'_l (c + 1/2). */
static double cell_angle(const orc_grid *g, int ax, int32_t c, int l)
{
    return g->wmin[ax] + g->dprime[ax][l] * ((double)c + 0.5);
}

/*
 * Exact rotational bound (not in the paper, which notes that its bound is not
 * strictly exact under rotation, Sec. III-D).  A level-l node is scored at the
 * centre rotation of its angular cell; a leaf below it has a rotation whose
 * angles differ from that centre by at most dev_ax per axis (the largest
 * distance between the node's cell centre and the centres of the leaf cells
 * [c P, (c + 1) P - 1], P the product of the divisions a of levels 1..l).
 * Since Rz Ry Rx changes by at most the sum of the three angle changes in
 * operator norm, a scan point moves by at most disp = d_max (dev_roll +
 * dev_pitch + dev_yaw), i.e. its level-0 voxel by at most
 * D = ceil((disp + slack) / r) per axis (slack = 1e-5 d_max + 1e-6 m covers
 * the float transform) and its level-l voxel by at most e_l = ceil(D / 2^l).
 * The node scored with the leaf's own rotation lands in D_l whenever the leaf
 * hits (the nesting of the translation-only case), so scoring the node against
 * D_l grown by [-e_l, e_l]^3 bounds every leaf below it.  Writes e_l to
 * out[l] for l = 1..levels (out[0] = 0; all 0 in translation-only mode, where
 * every node carries a leaf rotation).
 */
void orc_rotation_margins(const orc_grid *g, int32_t *out)
{
    for (int l = 0; l <= g->levels; ++l) out[l] = 0;
    if (g->translation_only) return;
    for (int l = 1; l <= g->levels; ++l) {
        double theta = 0.0;
        for (int ax = 0; ax < 3; ++ax) {
            int64_t P = 1;
            for (int j = 1; j <= l; ++j) P *= g->a[ax][j];
            double dev = 0.0;
            for (int32_t c = 0; c < g->n[ax][l]; ++c) {
                int64_t i0 = (int64_t)c * P, i1 = (int64_t)(c + 1) * P - 1;
                if (i0 > g->n[ax][0] - 1) break;
                if (i1 > g->n[ax][0] - 1) i1 = g->n[ax][0] - 1;
                double centre = cell_angle(g, ax, c, l);
                double d0 = fabs(cell_angle(g, ax, (int32_t)i0, 0) - centre);
                double d1 = fabs(cell_angle(g, ax, (int32_t)i1, 0) - centre);
                if (d0 > dev) dev = d0;
                if (d1 > dev) dev = d1;
            }
            theta += dev;
        }
        double disp = g->dmax * theta;
        double D = ceil((disp + 1e-5 * g->dmax + 1e-6) / (double)g->r);
        out[l] = (int32_t)ceil(D / ldexp(1.0, l));
    }
}

/* 1 when the map's grown tables cover every level's margin. */
static int margins_cover(const orc_map *m, const orc_grid *g)
{
    int32_t need[ORC_MAX_LEVELS];
    orc_rotation_margins(g, need);
    for (int l = 1; l <= g->levels; ++l)
        if (need[l] > 0 && (m->margin[l] < need[l] || !m->keys_rot[l])) return 0;
    return 1;
}

/*
 * Rotation of the pose's Euler angles (roll alpha, pitch beta, yaw gamma),
 * Sec. III-A.  Reading: R = Rz(gamma) Ry(beta) Rx(alpha), entries formed in
 * double with the products evaluated left to right, then rounded to float.
 */
static void euler_to_float_matrix(double al, double be, double ga, float R[9])
{
    double ca = cos(al), sa = sin(al);
    double cb = cos(be), sb = sin(be);
    double cg = cos(ga), sg = sin(ga);
    R[0] = (float)(cg * cb);
    R[1] = (float)(cg * sb * sa - sg * ca);
    R[2] = (float)(cg * sb * ca + sg * sa);
    R[3] = (float)(sg * cb);
    R[4] = (float)(sg * sb * sa + cg * ca);
    R[5] = (float)(sg * sb * ca - cg * sa);
    R[6] = (float)(-sb);
    R[7] = (float)(cb * sa);
    R[8] = (float)(cb * ca);
}

void orc_rotation(const orc_grid *g, int32_t level, int32_t ia, int32_t ib, int32_t ig, float R[9])
{
    euler_to_float_matrix(cell_angle(g, 0, ia, level), cell_angle(g, 1, ib, level),
                          cell_angle(g, 2, ig, level), R);
}

static int translation_valid(const orc_grid *g, int ax, int32_t c, int l)
{
    return c >= floor_div_pow2(g->lo[ax], l) && c <= floor_div_pow2(g->hi[ax], l);
}

static int node_valid(const orc_grid *g, int l, const int32_t t[3], const int32_t ang[3])
{
    for (int ax = 0; ax < 3; ++ax) {
        if (!translation_valid(g, ax, t[ax], l)) return 0;
        if (ang[ax] < 0 || ang[ax] >= g->n[ax][l]) return 0;
    }
    return 1;
}

/* ------------------------------------------------------------------ score (Eq. (12), Sec. III-C) */

/*
 * score(c) = sum_k H^{c_l}(T_{x_c} s_k).
 * The node's translation is x_c = r_l c (the 2D rule of Sec. III-B carried to
 * 3D).  Reading: the level-l voxel of R s_k + r_l c is computed as
 * floor(floor(float(R s_k) / r) / 2^l) + c, which equals
 * floor((R s_k + r_l c) / r_l) in exact arithmetic.
 */
int32_t orc_score(const orc_map *m, const float *scan, int64_t k, const orc_grid *g, int32_t level,
                  int32_t x, int32_t y, int32_t z, int32_t ia, int32_t ib, int32_t ig)
{
    float R[9];
    orc_rotation(g, level, ia, ib, ig, R);
    const float r = g->r;
    int32_t count = 0;
    const int grown = g->rot_exact && !g->translation_only && level > 0 && m->keys_rot[level];
    for (int64_t i = 0; i < k; ++i) {
        float sx = scan[3 * i], sy = scan[3 * i + 1], sz = scan[3 * i + 2];
        int32_t key[3];
        for (int row = 0; row < 3; ++row) {
            float t0 = R[3 * row + 0] * sx;
            float t1 = R[3 * row + 1] * sy;
            float t2 = R[3 * row + 2] * sz;
            float p = (t0 + t1) + t2;
            float q = p / r;
            key[row] = (int32_t)floorf(q);
        }
        int32_t vx = floor_div_pow2(key[0], level) + x;
        int32_t vy = floor_div_pow2(key[1], level) + y;
        int32_t vz = floor_div_pow2(key[2], level) + z;
        if (grown) count += set_contains(m->keys_rot[level], m->n_rot[level], vx, vy, vz);
        else count += orc_map_contains(m, level, vx, vy, vz);
    }
    return count;
}

/* nodes: n records of 7 int32 (level, x, y, z, roll, pitch, yaw) */
void orc_score_nodes(const orc_map *m, const float *scan, int64_t k, const orc_grid *g,
                     const int32_t *nodes, int64_t n, int32_t *scores, int32_t threads)
{
#pragma omp parallel for schedule(dynamic, 16) num_threads(threads > 0 ? threads : 1)
    for (int64_t i = 0; i < n; ++i) {
        const int32_t *c = nodes + 7 * i;
        scores[i] = orc_score(m, scan, k, g, c[0], c[1], c[2], c[3], c[4], c[5], c[6]);
    }
}

/* ------------------------------------------------------------------ search (Alg. 2) */

typedef struct {
    int32_t t[3], ang[3];
    int32_t level, score, parent_score;
    int64_t seq;
} orc_node;

typedef struct {
    orc_node *v;
    int64_t n, cap;
} node_vec;

static int vec_push(node_vec *q, const orc_node *x)
{
    if (q->n == q->cap) {
        int64_t cap = q->cap ? 2 * q->cap : 1024;
        orc_node *p = (orc_node *)realloc(q->v, (size_t)cap * sizeof(orc_node));
        if (!p) return ORC_ERR_OOM;
        q->v = p;
        q->cap = cap;
    }
    q->v[q->n++] = *x;
    return ORC_OK;
}

/*
 * Queue order.  Best-first search (Sec. III-D, Alg. 2) sorts C in descending
 * order of score; reading for ties: lower level first (the depth preference
 * of Alg. 1), then first-in first-out.  Depth-first search (Alg. 1, the
 * conventional BBS) keeps the queue sorted by depth level with the maximum
 * score popped first; reading: lower level first, then higher score, then
 * first-in first-out.
 */
enum { ORC_BEST_FIRST = 0, ORC_DEPTH_FIRST = 1 };

static int before(const orc_node *a, const orc_node *b, int order)
{
    if (order == ORC_DEPTH_FIRST && a->level != b->level) return a->level < b->level;
    if (a->score != b->score) return a->score > b->score;
    if (a->level != b->level) return a->level < b->level;
    return a->seq < b->seq;
}

static int heap_push(node_vec *h, const orc_node *x, int order)
{
    if (vec_push(h, x)) return ORC_ERR_OOM;
    int64_t i = h->n - 1;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (!before(&h->v[i], &h->v[p], order)) break;
        orc_node t = h->v[i]; h->v[i] = h->v[p]; h->v[p] = t;
        i = p;
    }
    return ORC_OK;
}

static orc_node heap_pop(node_vec *h, int order)
{
    orc_node top = h->v[0];
    h->v[0] = h->v[--h->n];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, m = i;
        if (l < h->n && before(&h->v[l], &h->v[m], order)) m = l;
        if (r < h->n && before(&h->v[r], &h->v[m], order)) m = r;
        if (m == i) break;
        orc_node t = h->v[i]; h->v[i] = h->v[m]; h->v[m] = t;
        i = m;
    }
    return top;
}

static int leaf_lex_less(const orc_node *a, const orc_node *b)
{
    for (int i = 0; i < 3; ++i) if (a->t[i] != b->t[i]) return a->t[i] < b->t[i];
    for (int i = 0; i < 3; ++i) if (a->ang[i] != b->ang[i]) return a->ang[i] < b->ang[i];
    return 0;
}

typedef struct {
    int32_t found, score;
    int32_t leaf[6];                 /* i_x, i_y, i_z, i_roll, i_pitch, i_yaw */
    double pose[6];                  /* x, y, z [m], roll, pitch, yaw [rad] */
    int64_t nodes_expanded;          /* accepted non-leaf pops (branched nodes) */
    int64_t nodes_scored;            /* initial set + every flushed child */
    int64_t flushes;                 /* batches sent to scoring */
    int64_t leaves_accepted;         /* leaf pops with score >= best */
    int64_t initial_size, initial_kept;
    int64_t bound_checks, bound_violations;  /* children scored / children above parent */
    double violation_excess_sum;             /* sum of (child - parent) / parent */
    int32_t prior_used, seeded;              /* the prior ordered the initial set; the seed beam set the incumbent */
    int32_t seed_score, pad;
    int64_t events;                          /* search events logged (see orc_localize) */
} orc_result;

/*
 * Children of node c (Sec. III-D, roto-translational branching):
 *   (2c_x + j_x, 2c_y + j_y, 2c_z + j_z, a_a c_a + j_a, a_b c_b + j_b, a_g c_g + j_g, l - 1).
 * Readings: enumeration with the rotational offsets outer (j_a, j_b, j_g in
 * lexicographic order) and the translational ones inner (j_x, j_y, j_z); a
 * child whose angle index reaches the level's cell count, or whose leaf
 * interval misses the translation range, is not generated.
 */
static int branch(const orc_grid *g, const orc_node *c, node_vec *pending)
{
    int l = c->level, cl = l - 1;
    int32_t ja[3];
    for (ja[0] = 0; ja[0] < g->a[0][l]; ++ja[0])
        for (ja[1] = 0; ja[1] < g->a[1][l]; ++ja[1])
            for (ja[2] = 0; ja[2] < g->a[2][l]; ++ja[2]) {
                orc_node ch;
                memset(&ch, 0, sizeof(ch));
                ch.level = cl;
                ch.parent_score = c->score;
                for (int ax = 0; ax < 3; ++ax) ch.ang[ax] = g->a[ax][l] * c->ang[ax] + ja[ax];
                for (int jx = 0; jx <= 1; ++jx)
                    for (int jy = 0; jy <= 1; ++jy)
                        for (int jz = 0; jz <= 1; ++jz) {
                            ch.t[0] = 2 * c->t[0] + jx;
                            ch.t[1] = 2 * c->t[1] + jy;
                            ch.t[2] = 2 * c->t[2] + jz;
                            if (!node_valid(g, cl, ch.t, ch.ang)) continue;
                            if (vec_push(pending, &ch)) return ORC_ERR_OOM;
                        }
            }
    return ORC_OK;
}

static void score_vec(const orc_map *m, const float *scan, int64_t k, const orc_grid *g, node_vec *v,
                      int32_t threads)
{
#pragma omp parallel for schedule(dynamic, 8) num_threads(threads > 0 ? threads : 1)
    for (int64_t i = 0; i < v->n; ++i) {
        orc_node *c = &v->v[i];
        c->score = orc_score(m, scan, k, g, c->level, c->t[0], c->t[1], c->t[2], c->ang[0], c->ang[1],
                             c->ang[2]);
    }
}

static void decode_pose(const orc_grid *g, const int32_t leaf[6], double pose[6])
{
    for (int ax = 0; ax < 3; ++ax) pose[ax] = (double)g->r * leaf[ax];
    for (int ax = 0; ax < 3; ++ax) pose[3 + ax] = cell_angle(g, ax, leaf[3 + ax], 0);
}

/* ------------------------------------------------------------------ learned prior (not in the paper)
 *
 * The prior is 1088 logits: 64 over yaw bins, then 32 x 32 over translation
 * cells of the search box (x outer).  A yaw bin is [2 pi b / 64, 2 pi (b+1) / 64)
 * after reducing the angle mod 2 pi; a translation cell splits each of the
 * x and y search intervals into 32 equal parts.
 *
 * The key of a node is the best yaw-bin logit over the leaf yaws below it
 * plus the best cell logit over the leaf translations below it.  The leaves
 * below a level-l node are the cells [c 2^l, (c+1) 2^l - 1] of each
 * translation axis (within the search range) and the yaw cells
 * [c P, (c+1) P - 1] with P the product of the yaw divisions a of levels
 * 1..l (within the level-0 cell count).  A key only orders nodes; it never
 * changes a score.
 */
#define ORC_YAW_BINS 64
#define ORC_XY_CELLS 32

static int yaw_bin_of(double th)
{
    const double two_pi = 2.0 * 3.14159265358979323846;
    double tm = th - two_pi * floor(th / two_pi);
    int yb = (int)floor(tm / (two_pi / ORC_YAW_BINS));
    if (yb < 0) yb = 0;
    if (yb >= ORC_YAW_BINS) yb = ORC_YAW_BINS - 1;
    return yb;
}

static int xy_cell_of(const orc_grid *g, int ax, int32_t i)
{
    double x = (double)g->r * (double)i;
    double lo = g->tmin[ax], hi = g->tmax[ax];
    int ci = hi > lo ? (int)floor(ORC_XY_CELLS * (x - lo) / (hi - lo)) : 0;
    if (ci < 0) ci = 0;
    if (ci >= ORC_XY_CELLS) ci = ORC_XY_CELLS - 1;
    return ci;
}

static double prior_key(const orc_grid *g, const float *prior, const orc_node *c)
{
    const int l = c->level;
    int64_t span = 1;
    for (int m = 1; m <= l; ++m) span *= g->a[2][m];
    int64_t y0 = (int64_t)c->ang[2] * span, y1 = ((int64_t)c->ang[2] + 1) * span - 1;
    if (y1 > g->n[2][0] - 1) y1 = g->n[2][0] - 1;
    double ky = -INFINITY;
    for (int64_t i = y0; i <= y1; ++i) {
        double v = prior[yaw_bin_of(cell_angle(g, 2, (int32_t)i, 0))];
        if (v > ky) ky = v;
    }
    uint32_t cells[2] = {0, 0};       /* bit c: some leaf below the node lies in cell c of this axis */
    for (int ax = 0; ax < 2; ++ax) {
        int64_t i0 = (int64_t)c->t[ax] << l, i1 = (((int64_t)c->t[ax] + 1) << l) - 1;
        if (i0 < g->lo[ax]) i0 = g->lo[ax];
        if (i1 > g->hi[ax]) i1 = g->hi[ax];
        for (int64_t i = i0; i <= i1; ++i) cells[ax] |= 1u << xy_cell_of(g, ax, (int32_t)i);
    }
    double kxy = -INFINITY;
    for (int cx = 0; cx < ORC_XY_CELLS; ++cx) {
        if (!((cells[0] >> cx) & 1u)) continue;
        for (int cy = 0; cy < ORC_XY_CELLS; ++cy) {
            if (!((cells[1] >> cy) & 1u)) continue;
            double v = prior[ORC_YAW_BINS + cx * ORC_XY_CELLS + cy];
            if (v > kxy) kxy = v;
        }
    }
    return ky + kxy;
}

/* node = (level, x, y, z, i_roll, i_pitch, i_yaw) */
double orc_prior_key(const orc_grid *g, const float *prior, const int32_t *node)
{
    orc_node c;
    memset(&c, 0, sizeof(c));
    c.level = node[0];
    for (int ax = 0; ax < 3; ++ax) {
        c.t[ax] = node[1 + ax];
        c.ang[ax] = node[4 + ax];
    }
    return prior_key(g, prior, &c);
}

typedef struct {
    double key;
    int64_t index;
} keyed;

static int cmp_keyed(const void *a, const void *b)
{
    const keyed *x = (const keyed *)a, *y = (const keyed *)b;
    if (x->key != y->key) return x->key > y->key ? -1 : 1;
    return (x->index > y->index) - (x->index < y->index);
}

/* beam candidates rank by score (desc), prior key (desc), position (asc) */
typedef struct {
    orc_node n;
    double key;
    int64_t pos;
} beam_item;

static int cmp_beam(const void *a, const void *b)
{
    const beam_item *x = (const beam_item *)a, *y = (const beam_item *)b;
    if (x->n.score != y->n.score) return x->n.score > y->n.score ? -1 : 1;
    if (x->key != y->key) return x->key > y->key ? -1 : 1;
    return (x->pos > y->pos) - (x->pos < y->pos);
}

/*
 * Seed beam: starting from the `width` best initial nodes (scored, at or
 * above the threshold; position = place in the prior order), branch every
 * beam node, score all children, and keep the `width` best children at or
 * above the threshold (position = place among the children, beam order then
 * branching order), down to the leaves.  The best beam leaf (highest score,
 * then lexicographically smallest) is returned.  Every branched beam node
 * counts as expanded and every child as scored.
 */
static int seed_beam(const orc_map *m, const float *scan, int64_t k, const orc_grid *g, const float *prior,
                     int32_t threshold, int32_t width, const node_vec *init, int32_t threads, orc_result *res,
                     orc_node *leaf, int *found)
{
    *found = 0;
    int rc = ORC_OK;
    node_vec ch = {0};
    beam_item *items = (beam_item *)malloc((size_t)(init->n ? init->n : 1) * sizeof(beam_item));
    if (!items) return ORC_ERR_OOM;
    int64_t n_items = 0, cap_items = init->n ? init->n : 1;
    for (int64_t i = 0; i < init->n; ++i) {
        if (init->v[i].score < threshold) continue;
        items[n_items].n = init->v[i];
        items[n_items].key = prior_key(g, prior, &init->v[i]);
        items[n_items].pos = i;
        ++n_items;
    }
    qsort(items, (size_t)n_items, sizeof(beam_item), cmp_beam);
    if (n_items > width) n_items = width;
    while (n_items > 0 && items[0].n.level > 0) {
        ch.n = 0;
        for (int64_t i = 0; i < n_items; ++i) {
            if ((rc = branch(g, &items[i].n, &ch))) goto out;
            res->nodes_expanded++;
        }
        score_vec(m, scan, k, g, &ch, threads);
        res->nodes_scored += ch.n;
        if (ch.n > cap_items) {
            beam_item *t = (beam_item *)realloc(items, (size_t)ch.n * sizeof(beam_item));
            if (!t) { rc = ORC_ERR_OOM; goto out; }
            items = t;
            cap_items = ch.n;
        }
        n_items = 0;
        for (int64_t i = 0; i < ch.n; ++i) {
            if (ch.v[i].score < threshold) continue;
            items[n_items].n = ch.v[i];
            items[n_items].key = prior_key(g, prior, &ch.v[i]);
            items[n_items].pos = i;
            ++n_items;
        }
        qsort(items, (size_t)n_items, sizeof(beam_item), cmp_beam);
        if (n_items > width) n_items = width;
    }
    for (int64_t i = 0; i < n_items; ++i) {
        const orc_node *c = &items[i].n;
        if (!*found || c->score > leaf->score || (c->score == leaf->score && leaf_lex_less(c, leaf))) {
            *leaf = *c;
            *found = 1;
        }
    }
out:
    free(items);
    free(ch.v);
    return rc;
}

/*
 * Batched best-first branch and bound, Alg. 2.
 *  - best_score starts at score_threshold; initial nodes below it are removed
 *    (Sec. III-D, search strategy).
 *  - pop c; skip it if its score is below best_score;
 *  - a leaf becomes the match and sets best_score.  Reading: among leaves of
 *    equal score the lexicographically smallest index (x, y, z, roll, pitch,
 *    yaw) is kept;
 *  - otherwise c is branched and its children are appended to the pending set;
 *  - when more than b nodes are pending they are scored and pushed.
 * Reading: when the queue runs empty while nodes are still pending, they are
 * scored and pushed too, so no branched child is lost.
 * Initial set (Sec. III-D: every pose in the search range at l_max).  Reading
 * for its order: the top-level cells are enumerated as the valid children of
 * virtual cells one level above, visited in lexicographic order, each
 * expanded like a branch (rotations outer, translations inner).
 * max_scored bounds the number of scored nodes (0 = no bound); a bounded run
 * returns found = -1 when it stops early.
 * With a finite prior (not in the paper) the initial set is scored and queued
 * in descending prior key (ties in enumeration order), and a seed beam of
 * width beam_width may set the incumbent before the loop starts.
 * order selects the search strategy: ORC_BEST_FIRST (Alg. 2, the paper's
 * proposal) or ORC_DEPTH_FIRST (the queue order of Alg. 1, Table I
 * configurations (a)-(c)); both use the batching, pruning and leaf rules
 * above, so that they differ in the pop order only.
 */
/* Event log of the search loop (tests only): 9 int32 per event, kind then the
 * node (level, x, y, z, roll, pitch, yaw) and its score.  Kinds: a popped node
 * that is pruned, an accepted leaf, a branched node; and a flush, whose
 * "score" field holds the number of nodes scored. */
enum { ORC_EV_PRUNE = 0, ORC_EV_LEAF = 1, ORC_EV_BRANCH = 2, ORC_EV_FLUSH = 3 };

static void log_event(int32_t *ev, int64_t cap, orc_result *res, int kind, const orc_node *c, int32_t value)
{
    if (ev && res->events < cap) {
        int32_t *e = ev + 9 * res->events;
        e[0] = kind;
        e[1] = c ? c->level : -1;
        for (int ax = 0; ax < 3; ++ax) {
            e[2 + ax] = c ? c->t[ax] : 0;
            e[5 + ax] = c ? c->ang[ax] : 0;
        }
        e[8] = value;
    }
    res->events++;
}

int orc_localize(const orc_map *m, const float *scan, int64_t k, const orc_grid *g, int32_t threshold,
                 int64_t batch, int32_t threads, int64_t max_scored, orc_result *res,
                 int64_t *trace_flush, int64_t trace_cap, const float *prior, int32_t beam_width,
                 int32_t *events, int64_t events_cap, int32_t order)
{
    memset(res, 0, sizeof(*res));
    if (!m || !scan || k < 1 || batch < 1 || g->levels != m->levels) return ORC_ERR_ARG;
    if (order != ORC_BEST_FIRST && order != ORC_DEPTH_FIRST) return ORC_ERR_ARG;
    if (g->rot_exact && !margins_cover(m, g)) return ORC_ERR_ARG;
    const int L = g->levels;
    node_vec heap = {0}, pending = {0};
    int64_t seq = 0;
    int32_t best = threshold;
    int have_match = 0;
    orc_node match;
    memset(&match, 0, sizeof(match));
    int rc = ORC_OK;

    /* initial set C_{l_max} */
    int32_t plo[3], phi[3];
    for (int ax = 0; ax < 3; ++ax) {
        plo[ax] = floor_div_pow2(g->lo[ax], L + 1);
        phi[ax] = floor_div_pow2(g->hi[ax], L + 1);
    }
    orc_node top;
    memset(&top, 0, sizeof(top));
    top.level = L;
    for (int32_t px = plo[0]; px <= phi[0]; ++px)
        for (int32_t py = plo[1]; py <= phi[1]; ++py)
            for (int32_t pz = plo[2]; pz <= phi[2]; ++pz)
                for (top.ang[0] = 0; top.ang[0] < g->n[0][L]; ++top.ang[0])
                    for (top.ang[1] = 0; top.ang[1] < g->n[1][L]; ++top.ang[1])
                        for (top.ang[2] = 0; top.ang[2] < g->n[2][L]; ++top.ang[2])
                            for (int jx = 0; jx <= 1; ++jx)
                                for (int jy = 0; jy <= 1; ++jy)
                                    for (int jz = 0; jz <= 1; ++jz) {
                                        top.t[0] = 2 * px + jx;
                                        top.t[1] = 2 * py + jy;
                                        top.t[2] = 2 * pz + jz;
                                        if (!node_valid(g, L, top.t, top.ang)) continue;
                                        if ((rc = vec_push(&pending, &top))) goto done;
                                    }
    if (prior) {
        int finite = 1;
        for (int i = 0; i < ORC_YAW_BINS + ORC_XY_CELLS * ORC_XY_CELLS; ++i) finite = finite && isfinite(prior[i]);
        if (finite) {
            keyed *kv = (keyed *)malloc((size_t)(pending.n ? pending.n : 1) * sizeof(keyed));
            orc_node *cp = (orc_node *)malloc((size_t)(pending.n ? pending.n : 1) * sizeof(orc_node));
            if (!kv || !cp) { free(kv); free(cp); rc = ORC_ERR_OOM; goto done; }
            for (int64_t i = 0; i < pending.n; ++i) {
                kv[i].key = prior_key(g, prior, &pending.v[i]);
                kv[i].index = i;
                cp[i] = pending.v[i];
            }
            qsort(kv, (size_t)pending.n, sizeof(keyed), cmp_keyed);
            for (int64_t i = 0; i < pending.n; ++i) pending.v[i] = cp[kv[i].index];
            free(kv);
            free(cp);
            res->prior_used = 1;
        }
    }
    score_vec(m, scan, k, g, &pending, threads);
    res->initial_size = pending.n;
    res->nodes_scored = pending.n;
    for (int64_t i = 0; i < pending.n; ++i) {
        if (pending.v[i].score < threshold) continue;
        pending.v[i].seq = seq++;
        if ((rc = heap_push(&heap, &pending.v[i], order))) goto done;
        res->initial_kept++;
    }
    if (res->prior_used && beam_width > 0) {
        orc_node leaf;
        int got = 0;
        if ((rc = seed_beam(m, scan, k, g, prior, threshold, beam_width, &pending, threads, res, &leaf, &got)))
            goto done;
        if (got && leaf.score >= best) {
            match = leaf;
            have_match = 1;
            best = leaf.score;
            res->seeded = 1;
            res->seed_score = leaf.score;
        }
    }
    pending.n = 0;

    for (;;) {
        if (max_scored > 0 && res->nodes_scored >= max_scored) { res->found = -1; goto done; }
        int flush = 0;
        if (heap.n == 0) {
            if (pending.n == 0) break;
            flush = 1;                                     /* termination flush */
        } else {
            orc_node c = heap_pop(&heap, order);
            if (c.score < best) {                          /* pruned */
                log_event(events, events_cap, res, ORC_EV_PRUNE, &c, c.score);
                continue;
            }
            if (c.level == 0) {
                log_event(events, events_cap, res, ORC_EV_LEAF, &c, c.score);
                res->leaves_accepted++;
                if (!have_match || c.score > best || leaf_lex_less(&c, &match)) match = c;
                have_match = 1;
                best = c.score;
            } else {
                log_event(events, events_cap, res, ORC_EV_BRANCH, &c, c.score);
                res->nodes_expanded++;
                if ((rc = branch(g, &c, &pending))) goto done;
            }
            if (pending.n > batch) flush = 1;
        }
        if (flush) {
            score_vec(m, scan, k, g, &pending, threads);
            if (trace_flush && res->flushes < trace_cap) trace_flush[res->flushes] = pending.n;
            log_event(events, events_cap, res, ORC_EV_FLUSH, NULL, (int32_t)pending.n);
            res->flushes++;
            res->nodes_scored += pending.n;
            for (int64_t i = 0; i < pending.n; ++i) {
                orc_node *ch = &pending.v[i];
                res->bound_checks++;
                if (ch->score > ch->parent_score) {
                    res->bound_violations++;
                    res->violation_excess_sum +=
                        (double)(ch->score - ch->parent_score) / (double)(ch->parent_score > 0 ? ch->parent_score : 1);
                }
                ch->seq = seq++;
                if ((rc = heap_push(&heap, ch, order))) goto done;
            }
            pending.n = 0;
        }
    }
    if (have_match) {
        res->found = 1;
        res->score = match.score;
        for (int ax = 0; ax < 3; ++ax) {
            res->leaf[ax] = match.t[ax];
            res->leaf[3 + ax] = match.ang[ax];
        }
        decode_pose(g, res->leaf, res->pose);
    }
done:
    free(heap.v);
    free(pending.v);
    return rc;
}

/*
 * Exhaustive search over the leaf set (the full search that branch and bound
 * must equal, Sec. III-B): argmax of the level-0 score over all valid leaves
 * with score >= threshold, ties to the lexicographically smallest index.
 */
int orc_bruteforce(const orc_map *m, const float *scan, int64_t k, const orc_grid *g, int32_t threshold,
                   int32_t threads, orc_result *res)
{
    memset(res, 0, sizeof(*res));
    int64_t nx = g->hi[0] - g->lo[0] + 1, ny = g->hi[1] - g->lo[1] + 1, nz = g->hi[2] - g->lo[2] + 1;
    int64_t na = g->n[0][0], nb = g->n[1][0], ng = g->n[2][0];
    int64_t total = nx * ny * nz * na * nb * ng;
    int32_t *sc = (int32_t *)malloc((size_t)total * sizeof(int32_t));
    if (!sc) return ORC_ERR_OOM;
#pragma omp parallel for schedule(dynamic, 64) num_threads(threads > 0 ? threads : 1)
    for (int64_t i = 0; i < total; ++i) {
        int64_t q = i;
        int32_t ig = (int32_t)(q % ng); q /= ng;
        int32_t ib = (int32_t)(q % nb); q /= nb;
        int32_t ia = (int32_t)(q % na); q /= na;
        int32_t z = (int32_t)(q % nz) + g->lo[2]; q /= nz;
        int32_t y = (int32_t)(q % ny) + g->lo[1]; q /= ny;
        int32_t x = (int32_t)q + g->lo[0];
        sc[i] = orc_score(m, scan, k, g, 0, x, y, z, ia, ib, ig);
    }
    int64_t arg = -1;
    int32_t best = threshold;
    for (int64_t i = 0; i < total; ++i)      /* row-major order is lexicographic order */
        if (sc[i] > best || (sc[i] == best && arg < 0)) { best = sc[i]; arg = i; }
    res->nodes_scored = total;
    if (arg >= 0) {
        int64_t q = arg;
        res->leaf[5] = (int32_t)(q % ng); q /= ng;
        res->leaf[4] = (int32_t)(q % nb); q /= nb;
        res->leaf[3] = (int32_t)(q % na); q /= na;
        res->leaf[2] = (int32_t)(q % nz) + g->lo[2]; q /= nz;
        res->leaf[1] = (int32_t)(q % ny) + g->lo[1]; q /= ny;
        res->leaf[0] = (int32_t)q + g->lo[0];
        res->found = 1;
        res->score = best;
        decode_pose(g, res->leaf, res->pose);
    }
    free(sc);
    return ORC_OK;
}

/* Score of every valid leaf in lexicographic order (tests on tiny grids). */
int64_t orc_all_leaf_scores(const orc_map *m, const float *scan, int64_t k, const orc_grid *g,
                            int32_t *out, int64_t cap, int32_t threads)
{
    int64_t nx = g->hi[0] - g->lo[0] + 1, ny = g->hi[1] - g->lo[1] + 1, nz = g->hi[2] - g->lo[2] + 1;
    int64_t na = g->n[0][0], nb = g->n[1][0], ng = g->n[2][0];
    int64_t total = nx * ny * nz * na * nb * ng;
    if (total > cap) return total;
#pragma omp parallel for schedule(dynamic, 64) num_threads(threads > 0 ? threads : 1)
    for (int64_t i = 0; i < total; ++i) {
        int64_t q = i;
        int32_t ig = (int32_t)(q % ng); q /= ng;
        int32_t ib = (int32_t)(q % nb); q /= nb;
        int32_t ia = (int32_t)(q % na); q /= na;
        int32_t z = (int32_t)(q % nz) + g->lo[2]; q /= nz;
        int32_t y = (int32_t)(q % ny) + g->lo[1]; q /= ny;
        int32_t x = (int32_t)q + g->lo[0];
        out[i] = orc_score(m, scan, k, g, 0, x, y, z, ia, ib, ig);
    }
    return total;
}

/* Children of one node, in the branching order used by orc_localize
 * (7 int32 per child: level, x, y, z, roll, pitch, yaw).  Returns the count. */
int64_t orc_children(const orc_grid *g, const int32_t *node, int32_t *out, int64_t cap)
{
    orc_node c;
    memset(&c, 0, sizeof(c));
    c.level = node[0];
    if (c.level < 1 || c.level > g->levels) return 0;
    for (int ax = 0; ax < 3; ++ax) { c.t[ax] = node[1 + ax]; c.ang[ax] = node[4 + ax]; }
    node_vec v = {0};
    if (branch(g, &c, &v)) { free(v.v); return -1; }
    int64_t n = v.n;
    for (int64_t i = 0; i < n && i < cap; ++i) {
        out[7 * i] = v.v[i].level;
        for (int ax = 0; ax < 3; ++ax) { out[7 * i + 1 + ax] = v.v[i].t[ax]; out[7 * i + 4 + ax] = v.v[i].ang[ax]; }
    }
    free(v.v);
    return n;
}

/* Size of the orc_grid and orc_result structs, so that the loader can check its layout. */
int64_t orc_sizeof_grid(void) { return (int64_t)sizeof(orc_grid); }
int64_t orc_sizeof_result(void) { return (int64_t)sizeof(orc_result); }

/*
 * CPU oracle for the neural shadow-mapping hot path -- TEST INFRASTRUCTURE.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  It shares no code with the GPU library: every
 * operation below is written out plainly, in the operation order that the
 * rasterisation and feature-gather specification fixes, so that a reader
 * can check it line by line against that specification.
 *
 * What it computes (paper: Sec. 3.1, "Supervised training pairs"):
 *   - a z-buffer rasteriser used for the light-view shadow map (the vanilla
 *     shadow-mapping pass, Sec. 1 and 3.1) and for the camera G-buffer;
 *   - the per-pixel feature gather: view depth d, normal n, emitter-to-
 *     occluder depth z, pixel-to-emitter depth z_f, emitter size r_e and
 *     their compositions (Sec. 3.1-3.2), plus the hard depth-test mask;
 *   - brute-force / BVH ray-cast visibility, emitter-to-receiver rays
 *     (supplemental Sec. 5 prefers emitter-to-scene rays), one ray for a
 *     point light and stratified samples over the emitter disk for a
 *     spherical light (Sec. 3.1 uses Monte-Carlo ray-traced targets).
 *
 * Build: gcc -O2 -std=c99 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC
 * (no contraction: every float/double product and sum is rounded separately).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define EMPTY_DEPTH 0x7F800000u          /* +inf bit pattern */
#define EMPTY_KEY 0xFFFFFFFFFFFFFFFFull

static uint32_t f2u(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }
static float u2f(uint32_t u) { float f; memcpy(&f, &u, 4); return f; }

/* ------------------------------------------------------------------ raster
 * mode 0: depth bits (uint32, min), cleared to +inf
 * mode 1: camera key (uint64 = depth_bits << 32 | triangle id, min), cleared to all-ones
 * mode 2: fragment count per texel (uint32), cleared to 0 (watertightness checks)
 * stats[0] = triangles dropped (w <= 1e-6 or outside the guard band),
 * stats[1] = zero-area triangles, stats[2] = fragments that passed the depth range.
 */
static void clip_vertex(const float *m, const float *p, float *c) {
    for (int r = 0; r < 4; ++r) {
        float acc = m[4 * r + 0] * p[0];
        acc = acc + m[4 * r + 1] * p[1];
        acc = acc + m[4 * r + 2] * p[2];
        c[r] = acc + m[4 * r + 3];
    }
}

static int64_t edge_fn(int64_t xa, int64_t ya, int64_t xb, int64_t yb, int64_t px, int64_t py) {
    return (xb - xa) * (py - ya) - (yb - ya) * (px - xa);
}

static int edge_inclusive(int64_t xa, int64_t ya, int64_t xb, int64_t yb) {
    int64_t dx = xb - xa, dy = yb - ya;
    return dy > 0 || (dy == 0 && dx < 0);
}

static int64_t floor_div(int64_t a, int64_t b) {   /* b > 0 */
    int64_t q = a / b;
    if ((a % b) != 0 && a < 0) q -= 1;
    return q;
}

int ora_raster(const float *tris, int n_tris, const float *m, int w, int h, int mode,
               void *out, long long *stats) {
    if (!tris || !m || !out || w <= 0 || h <= 0 || n_tris < 0) return 1;
    size_t npix = (size_t)w * (size_t)h;
    uint32_t *o32 = (uint32_t *)out;
    uint64_t *o64 = (uint64_t *)out;
    for (size_t k = 0; k < npix; ++k) {
        if (mode == 0) o32[k] = EMPTY_DEPTH;
        else if (mode == 1) o64[k] = EMPTY_KEY;
        else o32[k] = 0;
    }
    long long dropped = 0, degenerate = 0, frags = 0;
    const float fw = (float)w, fh = (float)h;
    for (int t = 0; t < n_tris; ++t) {
        float c[3][4];
        int drop = 0;
        for (int v = 0; v < 3; ++v) {
            clip_vertex(m, tris + 9 * t + 3 * v, c[v]);
            if (!(c[v][3] > 1e-6f)) drop = 1;
        }
        if (drop) { dropped++; continue; }
        int64_t X[3], Y[3];
        float Z[3];
        for (int v = 0; v < 3; ++v) {
            float nx = c[v][0] / c[v][3];
            float ny = c[v][1] / c[v][3];
            float nz = c[v][2] / c[v][3];
            float sx = (nx * 0.5f + 0.5f) * fw;
            float sy = (ny * 0.5f + 0.5f) * fh;
            if (!(sx >= -8.0f * fw && sx <= 9.0f * fw && sy >= -8.0f * fh && sy <= 9.0f * fh)) drop = 1;
            X[v] = (int64_t)rintf(sx * 256.0f);
            Y[v] = (int64_t)rintf(sy * 256.0f);
            Z[v] = nz;
        }
        if (drop) { dropped++; continue; }
        int64_t A = (X[1] - X[0]) * (Y[2] - Y[0]) - (Y[1] - Y[0]) * (X[2] - X[0]);
        if (A == 0) { degenerate++; continue; }
        if (A < 0) {
            int64_t tx = X[1]; X[1] = X[2]; X[2] = tx;
            int64_t ty = Y[1]; Y[1] = Y[2]; Y[2] = ty;
            float tz = Z[1]; Z[1] = Z[2]; Z[2] = tz;
            A = -A;
        }
        int64_t xmin = X[0], xmax = X[0], ymin = Y[0], ymax = Y[0];
        for (int v = 1; v < 3; ++v) {
            if (X[v] < xmin) xmin = X[v];
            if (X[v] > xmax) xmax = X[v];
            if (Y[v] < ymin) ymin = Y[v];
            if (Y[v] > ymax) ymax = Y[v];
        }
        int64_t i0 = floor_div(xmin - 128, 256), i1 = floor_div(xmax - 128, 256) + 1;
        int64_t j0 = floor_div(ymin - 128, 256), j1 = floor_div(ymax - 128, 256) + 1;
        if (i0 < 0) i0 = 0;
        if (j0 < 0) j0 = 0;
        if (i1 > w - 1) i1 = w - 1;
        if (j1 > h - 1) j1 = h - 1;
        int inc0 = edge_inclusive(X[1], Y[1], X[2], Y[2]);
        int inc1 = edge_inclusive(X[2], Y[2], X[0], Y[0]);
        int inc2 = edge_inclusive(X[0], Y[0], X[1], Y[1]);
        for (int64_t j = j0; j <= j1; ++j) {
            for (int64_t i = i0; i <= i1; ++i) {
                int64_t px = 256 * i + 128, py = 256 * j + 128;
                int64_t e0 = edge_fn(X[1], Y[1], X[2], Y[2], px, py);
                int64_t e1 = edge_fn(X[2], Y[2], X[0], Y[0], px, py);
                int64_t e2 = edge_fn(X[0], Y[0], X[1], Y[1], px, py);
                int in0 = e0 > 0 || (e0 == 0 && inc0);
                int in1 = e1 > 0 || (e1 == 0 && inc1);
                int in2 = e2 > 0 || (e2 == 0 && inc2);
                if (!(in0 && in1 && in2)) continue;
                size_t k = (size_t)j * (size_t)w + (size_t)i;
                if (mode == 2) { o32[k] += 1; continue; }
                double num = (double)e0 * (double)Z[0];
                num = num + (double)e1 * (double)Z[1];
                num = num + (double)e2 * (double)Z[2];
                float d = (float)(num / (double)A);
                if (!(d >= 0.0f && d <= 1.0f)) continue;
                uint32_t bits = f2u(d);
                if ((bits & 0x7FFFFFFFu) == 0) bits = 0;  /* -0 becomes +0 */
                frags++;
                if (mode == 0) {
                    if (bits < o32[k]) o32[k] = bits;
                } else {
                    uint64_t key = ((uint64_t)bits << 32) | (uint64_t)(uint32_t)t;
                    if (key < o64[k]) o64[k] = key;
                }
            }
        }
    }
    if (stats) { stats[0] = dropped; stats[1] = degenerate; stats[2] = frags; }
    return 0;
}

/* ------------------------------------------------------------------ gather
 * Frame parameter vector (float32), indices:
 *   0..15  light matrix (row-major)    16..18 light position      19 light radius r_e
 *   20 light near   21 light far      22 light tan(half fov)    23 shadow-map size S
 *   24..39 camera matrix               40..42 camera position
 *   43..45 camera forward  46..48 camera right  49..51 camera up
 *   52 tan(half fov x)  53 tan(half fov y)  54 camera near  55 camera far
 * Channels (NHWC, C = 6 hard or 8 soft):
 *   [d/f_C, n.x, n.y, n.z, (z - z_f)/f_L, z/f_L] (+ [r_e/0.2, z_blk/f_L])
 * aux (optional, 4 floats per pixel): z, z_f, beta, inside flag.
 * pos (optional, 3 floats per pixel): receiver position P.
 */
static float lin_depth(float q, float nl, float fl) {
    float num = nl * fl;
    float den = fl - q * (fl - nl);
    return num / den;
}

int ora_gather(const float *tris, const float *normals, int n_tris, const float *fp,
               const uint64_t *gbuf, const uint32_t *sm, int w, int h, int fs,
               float *feat, uint8_t *mask, float *pos, float *aux) {
    if (!tris || !normals || !fp || !gbuf || !sm || !feat || w <= 0 || h <= 0) return 1;
    /* fs: 0 = [d/f_C, n, (z - z_f)/f_L, z/f_L]; 1 = that + [r_e/0.2, z_blk/f_L];
     * 2 = [c_e + r_e/0.0625, z/z_f, (z - z_f)/f_L, c_c/d] (the paper's selected set,
     * emitter size as a DC offset on c_e on a 0..4 scale) */
    const int soft = fs == 1;
    const int C = fs == 1 ? 8 : (fs == 2 ? 4 : 6);
    const float *ml = fp + 0, *L = fp + 16;
    const float r_e = fp[19], nl = fp[20], fl = fp[21], tanl = fp[22];
    const int S = (int)fp[23];
    const float *E = fp + 40, *fw = fp + 43, *rt = fp + 46, *up = fp + 49;
    const float tanx = fp[52], tany = fp[53], fc = fp[55];
    const float tau = (2.0f * tanl) / (float)S;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
    for (int j = 0; j < h; ++j) {
        for (int i = 0; i < w; ++i) {
            size_t p = (size_t)j * (size_t)w + (size_t)i;
            float *f = feat + p * (size_t)C;
            uint64_t key = gbuf[p];
            for (int c = 0; c < C; ++c) f[c] = 0.0f;
            if (mask) mask[p] = 0;
            if (pos) { pos[3 * p] = 0.0f; pos[3 * p + 1] = 0.0f; pos[3 * p + 2] = 0.0f; }
            if (aux) { aux[4 * p] = 0.0f; aux[4 * p + 1] = 0.0f; aux[4 * p + 2] = 0.0f; aux[4 * p + 3] = 0.0f; }
            if (key == EMPTY_KEY) continue;                 /* background */
            uint32_t t = (uint32_t)(key & 0xFFFFFFFFu);
            if ((int)t >= n_tris) { bad++; continue; }
            /* receiver position: pixel-centre camera ray meets the triangle's plane (float64) */
            double ndcx = (2.0 * ((double)i + 0.5)) / (double)w - 1.0;
            double ndcy = (2.0 * ((double)j + 0.5)) / (double)h - 1.0;
            double ax = ndcx * (double)tanx, ay = ndcy * (double)tany;
            double D[3];
            for (int k = 0; k < 3; ++k) D[k] = ((double)fw[k] + ax * (double)rt[k]) + ay * (double)up[k];
            const float *V0 = tris + 9 * (size_t)t;
            const float *N = normals + 3 * (size_t)t;
            double num = (double)N[0] * ((double)V0[0] - (double)E[0]);
            num = num + (double)N[1] * ((double)V0[1] - (double)E[1]);
            num = num + (double)N[2] * ((double)V0[2] - (double)E[2]);
            double den = (double)N[0] * D[0];
            den = den + (double)N[1] * D[1];
            den = den + (double)N[2] * D[2];
            if (den == 0.0) continue;
            double tt = num / den;
            float P[3];
            for (int k = 0; k < 3; ++k) P[k] = (float)((double)E[k] + tt * D[k]);
            /* normal facing the camera; view depth along the camera axis */
            float n[3] = {N[0], N[1], N[2]};
            float vx = E[0] - P[0], vy = E[1] - P[1], vz = E[2] - P[2];
            float s = n[0] * vx + n[1] * vy;
            s = s + n[2] * vz;
            if (s < 0.0f) { n[0] = -n[0]; n[1] = -n[1]; n[2] = -n[2]; }
            float dv = (P[0] - E[0]) * fw[0] + (P[1] - E[1]) * fw[1];
            dv = dv + (P[2] - E[2]) * fw[2];
            /* light-space projection and shadow-map texel */
            float c[4];
            clip_vertex(ml, P, c);
            int inside = c[3] > 1e-6f;
            float zf = fl, z = fl;
            int ti = 0, tj = 0;
            if (inside) {
                float nx = c[0] / c[3], ny = c[1] / c[3], nz = c[2] / c[3];
                float sx = (nx * 0.5f + 0.5f) * (float)S;
                float sy = (ny * 0.5f + 0.5f) * (float)S;
                zf = lin_depth(nz, nl, fl);
                inside = sx >= 0.0f && sx < (float)S && sy >= 0.0f && sy < (float)S &&
                         nz >= 0.0f && nz <= 1.0f;
                if (inside) {
                    ti = (int)floorf(sx);
                    tj = (int)floorf(sy);
                    uint32_t b = sm[(size_t)tj * (size_t)S + (size_t)ti];
                    if (b == EMPTY_DEPTH) inside = 0;
                    else z = lin_depth(u2f(b), nl, fl);
                }
            }
            /* slope-scaled bias */
            float lx = L[0] - P[0], ly = L[1] - P[1], lz = L[2] - P[2];
            float ll = lx * lx + ly * ly;
            ll = ll + lz * lz;
            float len = sqrtf(ll);
            float hx = lx / len, hy = ly / len, hz = lz / len;
            float cl = n[0] * hx + n[1] * hy;
            cl = cl + n[2] * hz;
            float sn = sqrtf(fmaxf(1.0f - cl * cl, 0.0f));
            float tq = sn / fmaxf(cl, 1e-3f);
            float beta = (zf * tau) * (1.0f + 1.5f * fminf(tq, 10.0f));
            if (mask) mask[p] = (uint8_t)(inside && zf > z + beta);
            if (fs == 2) {
                float vv = vx * vx + vy * vy;
                vv = vv + vz * vz;
                float cc = n[0] * vx + n[1] * vy;      /* cosine with the view direction */
                cc = cc + n[2] * vz;
                cc = cc / sqrtf(vv);
                f[0] = cl + r_e / 0.0625f;
                f[1] = z / zf;
                f[2] = (z - zf) / fl;
                f[3] = cc / dv;
            } else {
                f[0] = dv / fc;
                f[1] = n[0];
                f[2] = n[1];
                f[3] = n[2];
                f[4] = (z - zf) / fl;
                f[5] = z / fl;
            }
            if (soft) {
                float zb = zf;
                if (inside) {
                    float thr = zf - beta, sum = 0.0f;
                    int cnt = 0;
                    for (int dj = -3; dj <= 3; ++dj) {
                        int jj = tj + dj;
                        if (jj < 0 || jj >= S) continue;
                        for (int di = -3; di <= 3; ++di) {
                            int ii = ti + di;
                            if (ii < 0 || ii >= S) continue;
                            uint32_t b = sm[(size_t)jj * (size_t)S + (size_t)ii];
                            if (b == EMPTY_DEPTH) continue;
                            float q = lin_depth(u2f(b), nl, fl);
                            if (q < thr) { sum = sum + q; cnt++; }
                        }
                    }
                    if (cnt > 0) zb = sum / (float)cnt;
                }
                f[6] = r_e / 0.2f;
                f[7] = zb / fl;
            }
            if (pos) { pos[3 * p] = P[0]; pos[3 * p + 1] = P[1]; pos[3 * p + 2] = P[2]; }
            if (aux) { aux[4 * p] = z; aux[4 * p + 1] = zf; aux[4 * p + 2] = beta; aux[4 * p + 3] = (float)inside; }
        }
    }
    return bad ? 2 : 0;
}

/* ---------------------------------------------------------------- ray cast
 * Moller-Trumbore (1997) segment test in float64, any hit with parameter
 * t in (eps, 1 - eps) along origin -> origin + dir, over a median-split AABB
 * BVH (identical answers to brute force, which is also exposed).
 */
typedef struct { double lo[3], hi[3]; int left, right, first, count; } bvh_node;

typedef struct {
    const float *tris;
    int *idx;
    bvh_node *nodes;
    int n_nodes;
} bvh;

static int seg_hits_tri(const float *T, const double *o, const double *d, double eps) {
    double v0[3], e1[3], e2[3], pv[3], tv[3], qv[3];
    for (int k = 0; k < 3; ++k) {
        v0[k] = T[k];
        e1[k] = (double)T[3 + k] - v0[k];
        e2[k] = (double)T[6 + k] - v0[k];
    }
    pv[0] = d[1] * e2[2] - d[2] * e2[1];
    pv[1] = d[2] * e2[0] - d[0] * e2[2];
    pv[2] = d[0] * e2[1] - d[1] * e2[0];
    double det = e1[0] * pv[0] + e1[1] * pv[1] + e1[2] * pv[2];
    if (det == 0.0) return 0;
    double inv = 1.0 / det;
    for (int k = 0; k < 3; ++k) tv[k] = o[k] - v0[k];
    double u = (tv[0] * pv[0] + tv[1] * pv[1] + tv[2] * pv[2]) * inv;
    if (u < 0.0 || u > 1.0) return 0;
    qv[0] = tv[1] * e1[2] - tv[2] * e1[1];
    qv[1] = tv[2] * e1[0] - tv[0] * e1[2];
    qv[2] = tv[0] * e1[1] - tv[1] * e1[0];
    double v = (d[0] * qv[0] + d[1] * qv[1] + d[2] * qv[2]) * inv;
    if (v < 0.0 || u + v > 1.0) return 0;
    double t = (e2[0] * qv[0] + e2[1] * qv[1] + e2[2] * qv[2]) * inv;
    return t > eps && t < 1.0 - eps;
}

static void tri_bounds(const float *T, double *lo, double *hi) {
    for (int k = 0; k < 3; ++k) {
        double a = T[k], b = T[3 + k], c = T[6 + k];
        lo[k] = fmin(a, fmin(b, c));
        hi[k] = fmax(a, fmax(b, c));
    }
}

static const float *g_sort_tris;
static int g_sort_axis;
static int cmp_centroid(const void *a, const void *b) {
    const float *ta = g_sort_tris + 9 * (size_t)(*(const int *)a);
    const float *tb = g_sort_tris + 9 * (size_t)(*(const int *)b);
    double ca = (double)ta[g_sort_axis] + ta[3 + g_sort_axis] + ta[6 + g_sort_axis];
    double cb = (double)tb[g_sort_axis] + tb[3 + g_sort_axis] + tb[6 + g_sort_axis];
    return (ca > cb) - (ca < cb);
}

static int bvh_build_rec(bvh *b, int first, int count) {
    int ni = b->n_nodes++;
    bvh_node *nd = &b->nodes[ni];
    for (int k = 0; k < 3; ++k) { nd->lo[k] = INFINITY; nd->hi[k] = -INFINITY; }
    for (int q = first; q < first + count; ++q) {
        double lo[3], hi[3];
        tri_bounds(b->tris + 9 * (size_t)b->idx[q], lo, hi);
        for (int k = 0; k < 3; ++k) {
            if (lo[k] < nd->lo[k]) nd->lo[k] = lo[k];
            if (hi[k] > nd->hi[k]) nd->hi[k] = hi[k];
        }
    }
    nd->first = first;
    nd->count = count;
    nd->left = nd->right = -1;
    if (count <= 4) return ni;
    int axis = 0;
    double ext = -1.0;
    for (int k = 0; k < 3; ++k)
        if (nd->hi[k] - nd->lo[k] > ext) { ext = nd->hi[k] - nd->lo[k]; axis = k; }
    g_sort_tris = b->tris;
    g_sort_axis = axis;
    qsort(b->idx + first, (size_t)count, sizeof(int), cmp_centroid);
    int half = count / 2;
    int l = bvh_build_rec(b, first, half);
    int r = bvh_build_rec(b, first + half, count - half);
    b->nodes[ni].left = l;
    b->nodes[ni].right = r;
    b->nodes[ni].count = 0;
    return ni;
}

static int box_hit(const bvh_node *nd, const double *o, const double *d) {
    double t0 = 0.0, t1 = 1.0;
    for (int k = 0; k < 3; ++k) {
        if (d[k] == 0.0) {
            if (o[k] < nd->lo[k] || o[k] > nd->hi[k]) return 0;
            continue;
        }
        double ta = (nd->lo[k] - o[k]) / d[k], tb = (nd->hi[k] - o[k]) / d[k];
        if (ta > tb) { double x = ta; ta = tb; tb = x; }
        if (ta > t0) t0 = ta;
        if (tb < t1) t1 = tb;
        if (t0 > t1) return 0;
    }
    return 1;
}

static int bvh_occluded(const bvh *b, const double *o, const double *d, double eps) {
    int stack[128];
    int sp = 0;
    stack[sp++] = 0;
    while (sp > 0) {
        const bvh_node *nd = &b->nodes[stack[--sp]];
        if (!box_hit(nd, o, d)) continue;
        if (nd->left < 0) {
            for (int q = nd->first; q < nd->first + nd->count; ++q)
                if (seg_hits_tri(b->tris + 9 * (size_t)b->idx[q], o, d, eps)) return 1;
        } else {
            stack[sp++] = nd->left;
            stack[sp++] = nd->right;
        }
    }
    return 0;
}

static uint64_t sm64_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static double sm64_uniform(uint64_t key, uint64_t counter) {
    uint64_t z = sm64_mix(key + (counter + 1) * 0x9E3779B97F4A7C15ull);
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

/* Shirley-Chiu concentric square-to-disk map of (a, b) in [0,1)^2. */
static void concentric_disk(double a, double b, double *x, double *y) {
    double sx = 2.0 * a - 1.0, sy = 2.0 * b - 1.0;
    if (sx == 0.0 && sy == 0.0) { *x = 0.0; *y = 0.0; return; }
    double r, phi;
    if (fabs(sx) > fabs(sy)) { r = sx; phi = (M_PI / 4.0) * (sy / sx); }
    else { r = sy; phi = (M_PI / 2.0) - (M_PI / 4.0) * (sx / sy); }
    *x = r * cos(phi);
    *y = r * sin(phi);
}

/* vis[p] = fraction of unoccluded emitter samples for receivers pos[p]
 * (only where valid[p] != 0; others get 1).  radius == 0 or samples == 1:
 * a single ray from the light centre.  Otherwise samples = s*s strata on the
 * disk of the given radius centred at the light, facing the receiver.
 * use_bvh == 0 tests every triangle (brute force). */
int ora_raycast(const float *tris, int n_tris, const float *pos, const uint8_t *valid, int npix,
                const float *light, float radius, int samples, uint64_t seed, int use_bvh,
                double eps, float *vis) {
    if (!tris || !pos || !vis || n_tris < 0 || npix < 0 || samples < 1) return 1;
    int s = (int)lround(sqrt((double)samples));
    if (s * s != samples) return 1;
    bvh b;
    b.tris = tris;
    b.idx = (int *)malloc(sizeof(int) * (size_t)(n_tris > 0 ? n_tris : 1));
    b.nodes = (bvh_node *)malloc(sizeof(bvh_node) * (size_t)(2 * n_tris + 2));
    b.n_nodes = 0;
    if (!b.idx || !b.nodes) { free(b.idx); free(b.nodes); return 3; }
    for (int q = 0; q < n_tris; ++q) b.idx[q] = q;
    if (use_bvh && n_tris > 0) bvh_build_rec(&b, 0, n_tris);
    const double Lc[3] = {light[0], light[1], light[2]};
#pragma omp parallel for schedule(dynamic, 256)
    for (int p = 0; p < npix; ++p) {
        if (valid && !valid[p]) { vis[p] = 1.0f; continue; }
        double P[3] = {pos[3 * p], pos[3 * p + 1], pos[3 * p + 2]};
        double wv[3] = {P[0] - Lc[0], P[1] - Lc[1], P[2] - Lc[2]};
        double wl = sqrt(wv[0] * wv[0] + wv[1] * wv[1] + wv[2] * wv[2]);
        for (int k = 0; k < 3; ++k) wv[k] /= wl;
        double ref[3] = {0.0, 1.0, 0.0};
        if (fabs(wv[1]) > 0.9) { ref[0] = 1.0; ref[1] = 0.0; }
        double u[3] = {wv[1] * ref[2] - wv[2] * ref[1], wv[2] * ref[0] - wv[0] * ref[2],
                       wv[0] * ref[1] - wv[1] * ref[0]};
        double ul = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        for (int k = 0; k < 3; ++k) u[k] /= ul;
        double v[3] = {wv[1] * u[2] - wv[2] * u[1], wv[2] * u[0] - wv[0] * u[2],
                       wv[0] * u[1] - wv[1] * u[0]};
        uint64_t key = sm64_mix(seed ^ ((uint64_t)p * 0x94D049BB133111EBull));
        int lit = 0;
        int nsamp = (radius > 0.0f && samples > 1) ? samples : 1;
        for (int q = 0; q < nsamp; ++q) {
            double o[3] = {Lc[0], Lc[1], Lc[2]};
            if (nsamp > 1) {
                double a = ((double)(q % s) + sm64_uniform(key, 2 * (uint64_t)q)) / (double)s;
                double bb = ((double)(q / s) + sm64_uniform(key, 2 * (uint64_t)q + 1)) / (double)s;
                double dx, dy;
                concentric_disk(a, bb, &dx, &dy);
                for (int k = 0; k < 3; ++k) o[k] += (double)radius * (dx * u[k] + dy * v[k]);
            }
            double d[3] = {P[0] - o[0], P[1] - o[1], P[2] - o[2]};
            int occ = 0;
            if (use_bvh && n_tris > 0) occ = bvh_occluded(&b, o, d, eps);
            else
                for (int t = 0; t < n_tris && !occ; ++t) occ = seg_hits_tri(tris + 9 * (size_t)t, o, d, eps);
            lit += !occ;
        }
        vis[p] = (float)((double)lit / (double)nsamp);
    }
    free(b.idx);
    free(b.nodes);
    return 0;
}

/* ------------------------------------------------------ temporal metric
 * Temporal instability of Eq. 3 for one pair of consecutive frames: the sum
 * over the current frame's pixels p of exp(alpha * D(p)) - 1, where
 * D(p) = |I_t(p) - I_{t-1}(m(p))| and m(p) is the motion-compensated pixel
 * of the previous frame.  Per pixel (i, j) of the current frame:
 *   1. background (empty key) -> no term;
 *   2. receiver P and camera-facing normal n of the current frame, as in
 *      the gather (float64 ray / plane intersection, rounded to float32);
 *   3. P projected with the previous camera matrix (float32, products and
 *      sums in the written order), c_w <= 1e-6 or outside the screen ->
 *      rejected; m(p) = (floor(sx), floor(sy));
 *   4. previous key at m(p) empty -> rejected;
 *   5. previous receiver P' and normal n' at m(p) (previous camera);
 *   6. depth test: view depths of P and P' along the previous camera axis,
 *      rejected when |dv - dv'| > depth_tol * dv';
 *   7. normal test: rejected when n . n' < cos_tol;
 *   8. D = |I_t(p) - I_{t-1}(m(p))|, term = exp(alpha D) - 1 (float64).
 * Outputs the float64 sum of the terms, the number of pixels that passed,
 * and optionally per pixel D or a negative code: -1 background,
 * -2 off-screen, -3 empty previous pixel, -4 depth, -5 normal.
 */
static int cam_receiver(const float *tris, const float *normals, int n_tris, const float *fp,
                        uint64_t key, int i, int j, int w, int h, float *P, float *n) {
    const float *E = fp + 40, *fw = fp + 43, *rt = fp + 46, *up = fp + 49;
    const float tanx = fp[52], tany = fp[53];
    if (key == EMPTY_KEY) return 0;
    uint32_t t = (uint32_t)(key & 0xFFFFFFFFu);
    if ((int)t >= n_tris) return 0;
    double ndcx = (2.0 * ((double)i + 0.5)) / (double)w - 1.0;
    double ndcy = (2.0 * ((double)j + 0.5)) / (double)h - 1.0;
    double ax = ndcx * (double)tanx, ay = ndcy * (double)tany;
    double D[3];
    for (int k = 0; k < 3; ++k) D[k] = ((double)fw[k] + ax * (double)rt[k]) + ay * (double)up[k];
    const float *V0 = tris + 9 * (size_t)t;
    const float *N = normals + 3 * (size_t)t;
    double num = (double)N[0] * ((double)V0[0] - (double)E[0]);
    num = num + (double)N[1] * ((double)V0[1] - (double)E[1]);
    num = num + (double)N[2] * ((double)V0[2] - (double)E[2]);
    double den = (double)N[0] * D[0];
    den = den + (double)N[1] * D[1];
    den = den + (double)N[2] * D[2];
    if (den == 0.0) return 0;
    double tt = num / den;
    for (int k = 0; k < 3; ++k) P[k] = (float)((double)E[k] + tt * D[k]);
    n[0] = N[0]; n[1] = N[1]; n[2] = N[2];
    float vx = E[0] - P[0], vy = E[1] - P[1], vz = E[2] - P[2];
    float s = n[0] * vx + n[1] * vy;
    s = s + n[2] * vz;
    if (s < 0.0f) { n[0] = -n[0]; n[1] = -n[1]; n[2] = -n[2]; }
    return 1;
}

static float view_depth(const float *fp, const float *P) {
    const float *E = fp + 40, *fw = fp + 43;
    float dv = (P[0] - E[0]) * fw[0] + (P[1] - E[1]) * fw[1];
    return dv + (P[2] - E[2]) * fw[2];
}

int ora_temporal(const float *tris, const float *normals, int n_tris, const float *fp_prev,
                 const float *fp_cur, const uint64_t *gbuf_prev, const uint64_t *gbuf_cur,
                 const float *vis_prev, const float *vis_cur, int w, int h, float alpha,
                 float depth_tol, float cos_tol, double *sum_out, int64_t *valid_out, float *d_out) {
    if (!tris || !normals || !fp_prev || !fp_cur || !gbuf_prev || !gbuf_cur || !vis_prev ||
        !vis_cur || !sum_out || !valid_out || w <= 0 || h <= 0)
        return 1;
    const float *mprev = fp_prev + 24;
    double total = 0.0;
    int64_t valid = 0;
    for (int j = 0; j < h; ++j) {
        for (int i = 0; i < w; ++i) {
            size_t p = (size_t)j * (size_t)w + (size_t)i;
            float code = -1.0f;
            float P[3], n[3], Pq[3], nq[3];
            if (cam_receiver(tris, normals, n_tris, fp_cur, gbuf_cur[p], i, j, w, h, P, n)) {
                float c[4];
                clip_vertex(mprev, P, c);
                code = -2.0f;
                if (c[3] > 1e-6f) {
                    float nx = c[0] / c[3], ny = c[1] / c[3];
                    float sx = (nx * 0.5f + 0.5f) * (float)w;
                    float sy = (ny * 0.5f + 0.5f) * (float)h;
                    if (sx >= 0.0f && sx < (float)w && sy >= 0.0f && sy < (float)h) {
                        int iq = (int)floorf(sx), jq = (int)floorf(sy);
                        size_t q = (size_t)jq * (size_t)w + (size_t)iq;
                        code = -3.0f;
                        if (cam_receiver(tris, normals, n_tris, fp_prev, gbuf_prev[q], iq, jq, w, h, Pq, nq)) {
                            float dv = view_depth(fp_prev, P), dq = view_depth(fp_prev, Pq);
                            float cs = n[0] * nq[0] + n[1] * nq[1];
                            cs = cs + n[2] * nq[2];
                            if (fabsf(dv - dq) > depth_tol * dq) code = -4.0f;
                            else if (cs < cos_tol) code = -5.0f;
                            else {
                                float D = fabsf(vis_cur[p] - vis_prev[q]);
                                total += exp((double)alpha * (double)D) - 1.0;
                                valid++;
                                code = D;
                            }
                        }
                    }
                }
            }
            if (d_out) d_out[p] = code;
        }
    }
    *sum_out = total;
    *valid_out = valid;
    return 0;
}

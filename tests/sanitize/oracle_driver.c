/* Command-line driver of the C oracle (oracle/nsm_oracle.c) for the
 * sanitizer test: it is linked with the oracle under AddressSanitizer and
 * UndefinedBehaviorSanitizer, reads every input array from a raw file into a
 * buffer of exactly the file's size, runs one oracle call, and writes every
 * output array to a raw file of exactly its size, so that any access past an
 * array, any misaligned or out-of-range integer operation, stops the run.
 *
 *   raster   tris n m w h mode out stats
 *   gather   tris normals n fp gbuf sm w h fs feat mask pos aux
 *   raycast  tris n pos valid|- npix light radius samples seed use_bvh eps vis
 *   temporal tris normals n fp_prev fp_cur gbuf_prev gbuf_cur vis_prev vis_cur w h alpha dtol ctol sum valid d
 *
 * Exit status: the oracle's return code, or 2 for a usage or I/O error. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int ora_raster(const float *tris, int n_tris, const float *m, int w, int h, int mode, void *out,
               long long *stats);
int ora_gather(const float *tris, const float *normals, int n_tris, const float *fp, const uint64_t *gbuf,
               const uint32_t *sm, int w, int h, int fs, float *feat, uint8_t *mask, float *pos, float *aux);
int ora_raycast(const float *tris, int n_tris, const float *pos, const uint8_t *valid, int npix,
                const float *light, float radius, int samples, uint64_t seed, int use_bvh, double eps,
                float *vis);
int ora_temporal(const float *tris, const float *normals, int n_tris, const float *fp_prev, const float *fp_cur,
                 const uint64_t *gbuf_prev, const uint64_t *gbuf_cur, const float *vis_prev,
                 const float *vis_cur, int w, int h, float alpha, float depth_tol, float cos_tol,
                 double *sum_out, int64_t *valid_out, float *d_out);

static void *read_all(const char *path) {
    if (strcmp(path, "-") == 0) return NULL;
    FILE *f = fopen(path, "rb");
    if (!f) { fprintf(stderr, "cannot open %s\n", path); exit(2); }
    fseek(f, 0, SEEK_END);
    long n = ftell(f);
    fseek(f, 0, SEEK_SET);
    void *p = malloc(n > 0 ? (size_t)n : 1);
    if (!p || (n > 0 && fread(p, 1, (size_t)n, f) != (size_t)n)) { fprintf(stderr, "cannot read %s\n", path); exit(2); }
    fclose(f);
    return p;
}

static void *alloc(size_t n) {
    void *p = malloc(n > 0 ? n : 1);
    if (!p) exit(2);
    return p;
}

static void write_all(const char *path, const void *p, size_t n) {
    FILE *f = fopen(path, "wb");
    if (!f || fwrite(p, 1, n, f) != n) { fprintf(stderr, "cannot write %s\n", path); exit(2); }
    fclose(f);
}

int main(int argc, char **argv) {
    if (argc < 2) return 2;
    const char *op = argv[1];
    int rc;
    if (strcmp(op, "raster") == 0 && argc == 10) {
        const int n = atoi(argv[3]), w = atoi(argv[5]), h = atoi(argv[6]), mode = atoi(argv[7]);
        const size_t bytes = (size_t)w * (size_t)h * (mode == 1 ? 8 : 4);
        void *out = alloc(bytes);
        long long *stats = alloc(3 * sizeof(long long));
        rc = ora_raster(read_all(argv[2]), n, read_all(argv[4]), w, h, mode, out, stats);
        write_all(argv[8], out, bytes);
        write_all(argv[9], stats, 3 * sizeof(long long));
    } else if (strcmp(op, "gather") == 0 && argc == 15) {
        const int n = atoi(argv[4]), w = atoi(argv[8]), h = atoi(argv[9]), fs = atoi(argv[10]);
        const int C = fs == 1 ? 8 : (fs == 2 ? 4 : 6);
        const size_t px = (size_t)w * (size_t)h;
        float *feat = alloc(px * C * 4), *pos = alloc(px * 12), *aux = alloc(px * 16);
        uint8_t *mask = alloc(px);
        rc = ora_gather(read_all(argv[2]), read_all(argv[3]), n, read_all(argv[5]), read_all(argv[6]),
                        read_all(argv[7]), w, h, fs, feat, mask, pos, aux);
        write_all(argv[11], feat, px * C * 4);
        write_all(argv[12], mask, px);
        write_all(argv[13], pos, px * 12);
        write_all(argv[14], aux, px * 16);
    } else if (strcmp(op, "raycast") == 0 && argc == 14) {
        const int n = atoi(argv[3]), npix = atoi(argv[6]), samples = atoi(argv[9]), use_bvh = atoi(argv[11]);
        float *vis = alloc((size_t)npix * 4);
        rc = ora_raycast(read_all(argv[2]), n, read_all(argv[4]), read_all(argv[5]), npix, read_all(argv[7]),
                         (float)atof(argv[8]), samples, strtoull(argv[10], NULL, 10), use_bvh, atof(argv[12]), vis);
        write_all(argv[13], vis, (size_t)npix * 4);
    } else if (strcmp(op, "temporal") == 0 && argc == 19) {
        const int n = atoi(argv[4]), w = atoi(argv[11]), h = atoi(argv[12]);
        double *sum = alloc(8);
        int64_t *valid = alloc(8);
        float *d = alloc((size_t)w * (size_t)h * 4);
        rc = ora_temporal(read_all(argv[2]), read_all(argv[3]), n, read_all(argv[5]), read_all(argv[6]),
                          read_all(argv[7]), read_all(argv[8]), read_all(argv[9]), read_all(argv[10]), w, h,
                          (float)atof(argv[13]), (float)atof(argv[14]), (float)atof(argv[15]), sum, valid, d);
        write_all(argv[16], sum, 8);
        write_all(argv[17], valid, 8);
        write_all(argv[18], d, (size_t)w * (size_t)h * 4);
    } else {
        fprintf(stderr, "usage error\n");
        return 2;
    }
    return rc;
}

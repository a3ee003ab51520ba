/* Runs the oracle's C entry points on one input file and writes every result
 * to an output file, so that a build under AddressSanitizer and
 * UndefinedBehaviorSanitizer can be compared with the normal library.
 *
 * Input (little-endian): int32 n_surf; per surface int64 nv, int64 nt,
 * int32 label, float center[3], float xyz[3 nv], int32 tri[3 nt]; int64 n;
 * float x[n], y[n], z[n]; double origin[3], double h, int64 cells[3];
 * int64 n_keys, uint64 keys[n_keys].
 * Output: int32 labels[n], double w[n_surf n], uint64 masks[n],
 * int32 radial_labels[n], uint64 radial_masks[n], int64 {lattice, keys
 * centroid, keys four-node} mismatches against all-zero labels, float
 * leaf points (rule 0, rule 1), double w0[n], uint8 on0[n], uint8 inside0[n]. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "sal_oracle.h"

static void *must(size_t bytes) {
    void *p = calloc(bytes ? bytes : 1, 1);
    if (!p) { fprintf(stderr, "out of memory\n"); exit(2); }
    return p;
}

static void rd(FILE *f, void *p, size_t bytes) {
    if (bytes && fread(p, 1, bytes, f) != bytes) { fprintf(stderr, "short input\n"); exit(2); }
}

static void wr(FILE *f, const void *p, size_t bytes) {
    if (bytes && fwrite(p, 1, bytes, f) != bytes) { fprintf(stderr, "short output\n"); exit(2); }
}

int main(int argc, char **argv) {
    if (argc != 3) { fprintf(stderr, "usage: oracle_driver in out\n"); return 2; }
    FILE *in = fopen(argv[1], "rb");
    if (!in) return 2;
    int32_t ns = 0;
    rd(in, &ns, 4);
    if (ns < 1 || ns > 64) return 2;
    int64_t *voff = must(sizeof(int64_t) * (ns + 1)), *toff = must(sizeof(int64_t) * (ns + 1));
    int32_t *labs = must(sizeof(int32_t) * ns);
    float *centers = must(sizeof(float) * 3 * ns);
    float **sv = must(sizeof(float *) * ns);
    int32_t **st = must(sizeof(int32_t *) * ns);
    int64_t *snv = must(sizeof(int64_t) * ns), *snt = must(sizeof(int64_t) * ns);
    for (int s = 0; s < ns; ++s) {
        rd(in, &snv[s], 8);
        rd(in, &snt[s], 8);
        rd(in, &labs[s], 4);
        rd(in, &centers[3 * s], 12);
        sv[s] = must(sizeof(float) * 3 * snv[s]);
        st[s] = must(sizeof(int32_t) * 3 * snt[s]);
        rd(in, sv[s], sizeof(float) * 3 * snv[s]);
        rd(in, st[s], sizeof(int32_t) * 3 * snt[s]);
        voff[s + 1] = voff[s] + snv[s];
        toff[s + 1] = toff[s] + snt[s];
    }
    float *verts = must(sizeof(float) * 3 * voff[ns]);
    int32_t *tris = must(sizeof(int32_t) * 3 * toff[ns]);
    for (int s = 0; s < ns; ++s) {
        memcpy(verts + 3 * voff[s], sv[s], sizeof(float) * 3 * snv[s]);
        memcpy(tris + 3 * toff[s], st[s], sizeof(int32_t) * 3 * snt[s]);
    }
    int64_t n = 0;
    rd(in, &n, 8);
    float *x = must(sizeof(float) * n), *y = must(sizeof(float) * n), *z = must(sizeof(float) * n);
    rd(in, x, sizeof(float) * n);
    rd(in, y, sizeof(float) * n);
    rd(in, z, sizeof(float) * n);
    double origin[3], h;
    int64_t cells[3], nk = 0;
    rd(in, origin, 24);
    rd(in, &h, 8);
    rd(in, cells, 24);
    rd(in, &nk, 8);
    uint64_t *keys = must(sizeof(uint64_t) * nk);
    rd(in, keys, sizeof(uint64_t) * nk);
    fclose(in);

    const int threads = 2;
    FILE *out = fopen(argv[2], "wb");
    if (!out) return 2;
    int32_t *lab = must(sizeof(int32_t) * n);
    double *w = must(sizeof(double) * ns * n);
    oracle_label(n, x, y, z, ns, voff, toff, verts, tris, labs, 0.5, threads, lab, w);
    wr(out, lab, sizeof(int32_t) * n);
    wr(out, w, sizeof(double) * ns * n);
    uint64_t *masks = must(sizeof(uint64_t) * n);
    oracle_enclosure(n, x, y, z, ns, voff, toff, verts, tris, 0.5, threads, masks);
    wr(out, masks, sizeof(uint64_t) * n);

    oracle_radial **rs = must(sizeof(oracle_radial *) * ns);
    for (int s = 0; s < ns; ++s) {
        int status = -1;
        rs[s] = oracle_radial_new(&centers[3 * s], snv[s], sv[s], snt[s], st[s], &status);
        if (!rs[s]) { fprintf(stderr, "radial index %d: status %d\n", s, status); return 3; }
    }
    int32_t *rlab = must(sizeof(int32_t) * n);
    uint64_t *rmask = must(sizeof(uint64_t) * n);
    if (oracle_radial_label(n, x, y, z, ns, rs, labs, threads, rlab, rmask) != 0) return 4;
    wr(out, rlab, sizeof(int32_t) * n);
    wr(out, rmask, sizeof(uint64_t) * n);

    const int64_t n_lat = 6 * cells[0] * cells[1] * cells[2];
    int32_t *zeros = must(sizeof(int32_t) * (n_lat > nk ? n_lat : nk));
    int64_t und = 0, bad[16], mism[3];
    mism[0] = oracle_radial_check_lattice(origin, h, cells, 0, n_lat, zeros, ns, rs, labs, threads,
                                          &und, bad, 16);
    mism[1] = oracle_radial_check_keys(origin, h, nk, keys, zeros, 0, ns, rs, labs, threads, &und,
                                       bad, 16);
    mism[2] = oracle_radial_check_keys(origin, h, nk, keys, zeros, 1, ns, rs, labs, threads, &und,
                                       bad, 16);
    if (und) return 5;
    wr(out, mism, sizeof(mism));
    float *lp = must(sizeof(float) * 12 * nk);
    oracle_leaf_points(origin, h, nk, keys, 0, lp);
    wr(out, lp, sizeof(float) * 3 * nk);
    oracle_leaf_points(origin, h, nk, keys, 1, lp);
    wr(out, lp, sizeof(float) * 12 * nk);

    double *w0 = must(sizeof(double) * n);
    uint8_t *on0 = must(n), *in0 = must(n);
    oracle_winding(n, x, y, z, snv[0], sv[0], snt[0], st[0], threads, w0, on0);
    oracle_radial_inside(n, x, y, z, &centers[0], sv[0], snt[0], st[0], threads, in0);
    wr(out, w0, sizeof(double) * n);
    wr(out, on0, n);
    wr(out, in0, n);
    fclose(out);

    for (int s = 0; s < ns; ++s) {
        oracle_radial_free(rs[s]);
        free(sv[s]);
        free(st[s]);
    }
    free(rs); free(sv); free(st); free(snv); free(snt); free(voff); free(toff); free(labs);
    free(centers); free(verts); free(tris); free(x); free(y); free(z); free(keys); free(lab);
    free(w); free(masks); free(rlab); free(rmask); free(zeros); free(lp); free(w0); free(on0);
    free(in0);
    return 0;
}

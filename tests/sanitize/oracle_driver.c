/*
 * The C oracle under the host sanitizers (AddressSanitizer and
 * UndefinedBehaviorSanitizer), linked into this program with lbm_oracle.c.
 * Usage: oracle_driver PARAMS_FILE F_FILE OUT_FILE NSTEPS
 *   PARAMS_FILE: the raw bytes of one oracle parameter block, as the tests'
 *     ctypes struct writes it (same compiler and ABI);
 *   F_FILE: 19 N doubles, the populations;
 *   OUT_FILE receives, back to back: oracle_step's 19 N doubles after NSTEPS
 *   steps; oracle_fields of the input (rho N, u 3N, F 3N, psi N, p N);
 *   oracle_collide_nodes of the first min(N, 64) nodes (19 each); and
 *   oracle_equilibrium of the input's rho with u = 0 (19 N).
 * Exit status 0 when every call returns 0.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

/* Entry points of lbm_oracle.c; the parameter block is opaque here. */
int oracle_step(const void *p, const double *fin, double *fout, int64_t nsteps);
int oracle_fields(const void *p, const double *f, double *rho, double *u, double *F, double *psi, double *pr);
int oracle_collide_nodes(const void *p, const double *f, int64_t count, const int64_t *idx, double *out);
int oracle_equilibrium(const void *p, const double *rho, const double *u, double *f);

static void *slurp(const char *path, long *size) {
    FILE *fh = fopen(path, "rb");
    if (!fh) return NULL;
    fseek(fh, 0, SEEK_END);
    *size = ftell(fh);
    fseek(fh, 0, SEEK_SET);
    void *buf = malloc((size_t)*size);
    if (buf && fread(buf, 1, (size_t)*size, fh) != (size_t)*size) {
        free(buf);
        buf = NULL;
    }
    fclose(fh);
    return buf;
}

int main(int argc, char **argv) {
    if (argc != 5) return 2;
    long psz = 0, fsz = 0;
    void *p = slurp(argv[1], &psz);
    double *f = (double *)slurp(argv[2], &fsz);
    if (!p || !f) return 3;
    const int32_t *dims = (const int32_t *)p;
    const int64_t N = (int64_t)dims[0] * dims[1] * dims[2];
    if (fsz != (long)(19 * N * (int64_t)sizeof(double))) return 4;
    const int64_t nsteps = atoll(argv[4]);
    const int64_t ns = N < 64 ? N : 64;
    double *step = malloc(sizeof(double) * 19 * N);
    double *fields = malloc(sizeof(double) * 9 * N);
    double *coll = malloc(sizeof(double) * 19 * ns);
    double *eq = malloc(sizeof(double) * 19 * N);
    double *zero_u = calloc((size_t)(3 * N), sizeof(double));
    int64_t *idx = malloc(sizeof(int64_t) * ns);
    if (!step || !fields || !coll || !eq || !zero_u || !idx) return 5;
    for (int64_t k = 0; k < ns; ++k) idx[k] = k;
    int rc = 0;
    rc |= oracle_step(p, f, step, nsteps);
    rc |= oracle_fields(p, f, fields, fields + N, fields + 4 * N, fields + 7 * N, fields + 8 * N);
    rc |= oracle_collide_nodes(p, f, ns, idx, coll);
    rc |= oracle_equilibrium(p, fields, zero_u, eq);
    FILE *out = fopen(argv[3], "wb");
    if (!out) return 6;
    fwrite(step, sizeof(double), (size_t)(19 * N), out);
    fwrite(fields, sizeof(double), (size_t)(9 * N), out);
    fwrite(coll, sizeof(double), (size_t)(19 * ns), out);
    fwrite(eq, sizeof(double), (size_t)(19 * N), out);
    fclose(out);
    free(step);
    free(fields);
    free(coll);
    free(eq);
    free(zero_u);
    free(idx);
    free(f);
    free(p);
    return rc ? 7 : 0;
}

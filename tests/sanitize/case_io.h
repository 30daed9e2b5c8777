/* Binary case files for the sanitizer drivers (test infrastructure): the
 * inputs of one oracle or host-mirror call, written by tests/test_sanitizers.py.
 *   int32 kind      1 pairs (op), 2 r2n (nr), 3 three-index overlap
 *   int32 arg       operator code or n of r_a^{2n} (unused for kind 3)
 *   int32 deriv     nonzero: d/dR_a blocks too
 *   double omega
 *   shells          (kind 3: orbital shells, then auxiliary shells)
 *   int64 n; int32 index[n][2 or 3]; int64 out_off[n]; int64 total
 * shells: int32 nshell; int64 nprim_total; double center[nshell][3];
 *         int32 l[nshell]; int32 nprim[nshell]; int64 prim_off[nshell];
 *         double exps[nprim_total]; double coefs[nprim_total]
 * The driver writes out[total] and, with deriv, dout[3 total] (doubles) to
 * the output file. Every array is exactly sized, so an access outside it is
 * caught by AddressSanitizer. */
#ifndef SHG_CASE_IO_H
#define SHG_CASE_IO_H
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    int32_t n;
    int64_t np;
    double *center;
    int32_t *l, *nprim;
    int64_t *prim_off;
    double *exps, *coefs;
} case_shells;

typedef struct {
    int32_t kind, arg, deriv;
    double omega;
    case_shells a, x;
    int64_t n, total;
    int32_t *idx;
    int64_t *out_off;
} case_t;

static void *case_read(FILE *f, size_t bytes)
{
    void *p = malloc(bytes ? bytes : 1);
    if (!p || (bytes && fread(p, 1, bytes, f) != bytes)) {
        fprintf(stderr, "case file truncated\n");
        exit(2);
    }
    return p;
}

static void case_read_shells(FILE *f, case_shells *s)
{
    int32_t *n = (int32_t *)case_read(f, sizeof(int32_t));
    int64_t *np = (int64_t *)case_read(f, sizeof(int64_t));
    s->n = *n;
    s->np = *np;
    free(n);
    free(np);
    s->center = (double *)case_read(f, sizeof(double) * 3 * (size_t)s->n);
    s->l = (int32_t *)case_read(f, sizeof(int32_t) * (size_t)s->n);
    s->nprim = (int32_t *)case_read(f, sizeof(int32_t) * (size_t)s->n);
    s->prim_off = (int64_t *)case_read(f, sizeof(int64_t) * (size_t)s->n);
    s->exps = (double *)case_read(f, sizeof(double) * (size_t)s->np);
    s->coefs = (double *)case_read(f, sizeof(double) * (size_t)s->np);
}

static void case_free_shells(case_shells *s)
{
    free(s->center);
    free(s->l);
    free(s->nprim);
    free(s->prim_off);
    free(s->exps);
    free(s->coefs);
}

static void case_load(const char *path, case_t *c)
{
    FILE *f = fopen(path, "rb");
    if (!f) {
        fprintf(stderr, "cannot open %s\n", path);
        exit(2);
    }
    int32_t *h = (int32_t *)case_read(f, 3 * sizeof(int32_t));
    c->kind = h[0];
    c->arg = h[1];
    c->deriv = h[2];
    free(h);
    double *w = (double *)case_read(f, sizeof(double));
    c->omega = *w;
    free(w);
    case_read_shells(f, &c->a);
    if (c->kind == 3) case_read_shells(f, &c->x);
    int64_t *n = (int64_t *)case_read(f, sizeof(int64_t));
    c->n = *n;
    free(n);
    const int width = c->kind == 3 ? 3 : 2;
    c->idx = (int32_t *)case_read(f, sizeof(int32_t) * (size_t)width * (size_t)c->n);
    c->out_off = (int64_t *)case_read(f, sizeof(int64_t) * (size_t)c->n);
    int64_t *t = (int64_t *)case_read(f, sizeof(int64_t));
    c->total = *t;
    free(t);
    fclose(f);
}

static void case_free(case_t *c)
{
    case_free_shells(&c->a);
    if (c->kind == 3) case_free_shells(&c->x);
    free(c->idx);
    free(c->out_off);
}

static void case_write(const char *path, const double *out, const double *dout, int64_t total)
{
    FILE *f = fopen(path, "wb");
    if (!f) {
        fprintf(stderr, "cannot write %s\n", path);
        exit(2);
    }
    fwrite(out, sizeof(double), (size_t)total, f);
    if (dout) fwrite(dout, sizeof(double), 3 * (size_t)total, f);
    fclose(f);
}
#endif

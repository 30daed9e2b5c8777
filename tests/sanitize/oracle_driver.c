/* Runs one CPU-oracle call on a case file (case_io.h) so that a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer checks the oracle's memory
 * accesses and arithmetic (test infrastructure).
 * usage: oracle_driver CASE OUT */
#include "case_io.h"

int shgo_pairs(int32_t nshell, const double *center, const int32_t *l, const int32_t *nprim,
               const int64_t *prim_off, const double *exps, const double *coefs, int op, double omega,
               const int32_t *pairs, int64_t n, const int64_t *out_off, double *out, double *dout);
int shgo_r2n(int32_t nshell, const double *center, const int32_t *l, const int32_t *nprim,
             const int64_t *prim_off, const double *exps, const double *coefs, int nr, const int32_t *pairs,
             int64_t n, const int64_t *out_off, double *out, double *dout);
int shgo_aab(int32_t norb, const double *oc, const int32_t *ol, const int32_t *onp, const int64_t *ooff,
             const double *oexp, const double *ocoef, int32_t naux, const double *xc, const int32_t *xl,
             const int32_t *xnp, const int64_t *xoff, const double *xexp, const double *xcoef,
             const int32_t *tri, int64_t n, const int64_t *out_off, double *out, double *dout);

int main(int argc, char **argv)
{
    if (argc != 3) {
        fprintf(stderr, "usage: %s CASE OUT\n", argv[0]);
        return 2;
    }
    case_t c;
    case_load(argv[1], &c);
    double *out = (double *)calloc((size_t)c.total + 1, sizeof(double));
    double *dout = c.deriv ? (double *)calloc(3 * (size_t)c.total + 1, sizeof(double)) : NULL;
    const case_shells *a = &c.a, *x = &c.x;
    int rc;
    if (c.kind == 1)
        rc = shgo_pairs(a->n, a->center, a->l, a->nprim, a->prim_off, a->exps, a->coefs, c.arg, c.omega, c.idx,
                        c.n, c.out_off, out, dout);
    else if (c.kind == 2)
        rc = shgo_r2n(a->n, a->center, a->l, a->nprim, a->prim_off, a->exps, a->coefs, c.arg, c.idx, c.n,
                      c.out_off, out, dout);
    else
        rc = shgo_aab(a->n, a->center, a->l, a->nprim, a->prim_off, a->exps, a->coefs, x->n, x->center, x->l,
                      x->nprim, x->prim_off, x->exps, x->coefs, c.idx, c.n, c.out_off, out, dout);
    if (rc == 0) case_write(argv[2], out, dout, c.total);
    else fprintf(stderr, "oracle call failed (%d)\n", rc);
    free(out);
    free(dout);
    case_free(&c);
    return rc == 0 ? 0 : 3;
}

// Runs one host-mirror call (the engine's device arithmetic compiled for the
// CPU) on a case file (case_io.h) so that a build with AddressSanitizer and
// UndefinedBehaviorSanitizer checks it (test infrastructure). Kind 1 only;
// the build instantiates the classes l_a, l_b <= 2 with derivatives (values
// come with them), and a pair of another class makes the call fail.
// usage: mirror_driver CASE OUT
#include "case_io.h"

extern "C" int shgm_pairs(int32_t nshell, const double *center, const int32_t *l, const int32_t *nprim,
                          const int64_t *prim_off, const double *exps, const double *coefs, int op,
                          double omega, const int32_t *pairs, int64_t n, const int64_t *out_off,
                          double *out, double *dout);

int main(int argc, char **argv)
{
    if (argc != 3) {
        fprintf(stderr, "usage: %s CASE OUT\n", argv[0]);
        return 2;
    }
    case_t c;
    case_load(argv[1], &c);
    if (c.kind != 1) {
        fprintf(stderr, "the host mirror has no entry for kind %d\n", c.kind);
        return 2;
    }
    double *out = (double *)calloc((size_t)c.total + 1, sizeof(double));
    double *dout = c.deriv ? (double *)calloc(3 * (size_t)c.total + 1, sizeof(double)) : nullptr;
    const case_shells *a = &c.a;
    const int rc = shgm_pairs(a->n, a->center, a->l, a->nprim, a->prim_off, a->exps, a->coefs, c.arg, c.omega,
                              c.idx, c.n, c.out_off, out, dout);
    if (rc == 0) case_write(argv[2], out, dout, c.total);
    else fprintf(stderr, "host-mirror call failed (%d)\n", rc);
    free(out);
    free(dout);
    case_free(&c);
    return rc == 0 ? 0 : 3;
}

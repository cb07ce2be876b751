/* Drives the FP64 oracle through every geometry kind and wall type for a few
 * steps, the moments, the observables and the stationarity check, built with
 * AddressSanitizer and UndefinedBehaviorSanitizer by
 * tests/test_native_sanitizers.py.  Exits 0 when every run stays finite. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    int kind, n1, n2, n3, walls, forcing_mode;
    double r_inner, width, b, tau, force, dtheta;
} orc_case;
typedef struct orc_sim orc_sim;
orc_sim *orc_create(const orc_case *cs, const double *init_u);
void orc_destroy(orc_sim *S);
void orc_step(orc_sim *S, long nsteps);
void orc_moments(const orc_sim *S, double *rho, double *u, double *lat_u);
void orc_observables(const orc_sim *S, double *omega_mean, double *v_mean, double *De);
double orc_check(orc_sim *S, int *bad);
void orc_get_f(const orc_sim *S, double *out_qn);

int main(void)
{
    const orc_case cases[] = {
        {0, 5, 2, 7, 5, 0, 1.0, 1.0, 1.0, 0.7, 1e-3, 0.0},   /* flat, walls on axes 1 and 3 */
        {1, 8, 3, 6, 1, 1, 1.0, 0.111, 1.0, 0.8, 1e-2, 0.0}, /* cylinder, old forcing       */
        {1, 9, 2, 6, 9, 0, 1.0, 0.111, 1.0, 0.9, 1e-2, 0.0}, /* cylinder, equilibrium walls */
        {2, 6, 2, 10, 1, 0, 10.0, 1.0, 1.4, 0.7, 1e-4, 0.0}, /* ellipsoid slab              */
        {3, 8, 12, 6, 1, 0, 3.0, 1.0, 1.4, 0.8, 1e-3, 0.0},  /* full ellipsoid              */
        {0, 4, 2, 4, 4, 0, 1.0, 1.0, 1.0, 0.75, 1e-3, 0.0},  /* walled axis 3 of 4 nodes    */
    };
    const int ncase = (int)(sizeof(cases) / sizeof(cases[0]));
    for (int k = 0; k < ncase; ++k) {
        const orc_case *c = &cases[k];
        const long N = (long)c->n1 * c->n2 * c->n3;
        double *u0 = calloc(3 * N, sizeof(double));
        for (long i = 0; i < 3 * N; ++i) u0[i] = 1e-3 * sin(0.37 * (double)i);
        orc_sim *S = orc_create(c, u0);
        orc_step(S, 7);
        int bad = 0;
        (void)orc_check(S, &bad);
        orc_step(S, 3);
        double r = orc_check(S, &bad);
        double *rho = malloc(sizeof(double) * N), *u = malloc(sizeof(double) * 3 * N);
        double *f = malloc(sizeof(double) * 41 * N);
        orc_moments(S, rho, u, NULL);
        orc_get_f(S, f);
        double om, vm, De;
        orc_observables(S, &om, &vm, &De);
        int finite = isfinite(r) && isfinite(om) && isfinite(vm) && isfinite(De) && !bad;
        for (long i = 0; i < 41 * N; ++i) finite &= isfinite(f[i]);
        printf("case %d: residual %.3e <omega> %.3e <v> %.3e De %.3e %s\n", k, r, om, vm, De, finite ? "ok" : "NOT FINITE");
        orc_destroy(S);
        free(u0); free(rho); free(u); free(f);
        if (!finite) return 1;
    }
    return 0;
}

/* Driver for the sanitizer test of the oracle (tests/test_oracle_sanitizers.py):
 * built together with oracle/clbm_oracle.c under AddressSanitizer and
 * UndefinedBehaviorSanitizer, it calls every lattice-level entry point of the
 * oracle on small lattices with walls, solid nodes, force fields, moving walls
 * and windows, and exits 0 when every call succeeds (with finite results on whole lattices).  Any
 * out-of-bounds access or undefined operation aborts the run. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int orc_init(const int *geom, const double *rho0, const double *u0, double *f);
int orc19_init(const int *geom, const double *rho0, const double *u0, double *f);
int orc_mrt_init(const int *geom, const double *rho0, const double *u0, double *f);
int orc_step(const int *geom, const double *s, const double *Fu, const double *Ff, const uint8_t *solid,
             const double *fin, double *fout);
int orc19_step(const int *geom, const double *s, const double *Fu, const double *Ff, const uint8_t *solid,
               const double *fin, double *fout);
int orc19_step_ex(const int *geom, const double *s, const double *Fu, const double *Ff, const uint8_t *solid,
                  const double *wall_u, const double *fin, double *fout);
int orc_step_ex(const int *geom, const double *s, const double *Fu, const double *Ff, const uint8_t *solid,
                const double *wall_u, int model, const double *fin, double *fout);
int orc_macro(const int *geom, const double *Fu, const double *Ff, const uint8_t *solid, const double *f,
              double *rho, double *u);
int orc19_macro(const int *geom, const double *Fu, const double *Ff, const uint8_t *solid, const double *f,
                double *rho, double *u);
int orc_adjoint_step(const int *geom, const double *s, const double *Fu, const double *Ff, const uint8_t *solid,
                     const double *f_t, const double *lam_next, double *lam_out, double *gF, double *gs);
int orc_loss_seed(const int *geom, const double *Fu, const double *Ff, const uint8_t *solid, const double *f,
                  const double *u_target, double *lam, double *gF, double *J);

static unsigned seed = 1801u;
static double rnd(void) /* uniform in [-0.5, 0.5) */
{
    seed = seed * 1103515245u + 12345u;
    return (double)((seed >> 8) & 0xffffu) / 65536.0 - 0.5;
}

static int failures = 0;
static void check(int rc, const char *what)
{
    if (rc != 0) {
        fprintf(stderr, "%s returned %d\n", what, rc);
        ++failures;
    }
}
/* A window is stepped with NaN pulled from outside it (its edge nodes depend on nodes it does not
 * hold), so its values are only checked by the sanitizers. */
static int full_lattice = 1;
static void check_finite(const double *a, long n, const char *what)
{
    if (!full_lattice) return;
    for (long i = 0; i < n; ++i)
        if (!isfinite(a[i])) {
            fprintf(stderr, "%s: non-finite value at %ld\n", what, i);
            ++failures;
            return;
        }
}

static double *alloc(long n)
{
    double *p = (double *)malloc(sizeof(double) * (size_t)n);
    if (!p) {
        fprintf(stderr, "out of memory\n");
        exit(2);
    }
    return p;
}

/* One lattice: geom = {nx, ny, nz, walls x y z, origin x y z, window x y z}. */
static void run_case(const int *geom, int with_solids, int with_field)
{
    const long nw = (long)geom[9] * geom[10] * geom[11];
    full_lattice = geom[9] == geom[0] && geom[10] == geom[1] && geom[11] == geom[2];
    const double s[10] = {1.0, 1.0, 1.6, 1.2, 1.3, 0.9, 1.1, 1.25, 0.95, 1.05};
    const double Fu[3] = {1e-5, -2e-6, 3e-6};
    double wall_u[18];
    for (int i = 0; i < 18; ++i) wall_u[i] = geom[3 + i / 6] ? 0.05 * rnd() : 0.0;
    double *rho0 = alloc(nw), *u0 = alloc(3 * nw), *Ff = alloc(3 * nw), *ut = alloc(3 * nw);
    uint8_t *solid = (uint8_t *)malloc((size_t)nw);
    for (long i = 0; i < nw; ++i) {
        rho0[i] = 1.0 + 0.02 * rnd();
        solid[i] = with_solids && rnd() < -0.35 ? 1 : 0;
    }
    for (long i = 0; i < 3 * nw; ++i) {
        u0[i] = 0.05 * rnd();
        Ff[i] = 1e-4 * rnd();
        ut[i] = 1e-3 * rnd();
    }
    const double *F = with_field ? Ff : NULL;
    const uint8_t *sol = with_solids ? solid : NULL;
    double *f = alloc(27 * nw), *g = alloc(27 * nw), *lam = alloc(27 * nw), *lam2 = alloc(27 * nw);
    double *rho = alloc(nw), *u = alloc(3 * nw), *gF = alloc(3 * nw), gs[10] = {0}, J = 0.0;
    for (long i = 0; i < 3 * nw; ++i) gF[i] = 0.0;

    /* D3Q27 cascaded, with and without moving walls, and the MRT */
    check(orc_init(geom, rho0, u0, f), "orc_init");
    check(orc_step(geom, s, Fu, F, sol, f, g), "orc_step");
    check(orc_step_ex(geom, s, Fu, F, sol, wall_u, 0, g, f), "orc_step_ex cascaded");
    check(orc_macro(geom, Fu, F, sol, f, rho, u), "orc_macro");
    check_finite(f, 27 * nw, "cascaded state");
    check_finite(u, 3 * nw, "velocity");
    check(orc_mrt_init(geom, rho0, u0, g), "orc_mrt_init");
    check(orc_step_ex(geom, s, Fu, F, sol, wall_u, 1, g, lam), "orc_step_ex mrt");
    check_finite(lam, 27 * nw, "mrt state");

    /* adjoint: loss seed and two reverse steps */
    check(orc_loss_seed(geom, Fu, F, sol, f, ut, lam, gF, &J), "orc_loss_seed");
    check(orc_adjoint_step(geom, s, Fu, F, sol, f, lam, lam2, gF, gs), "orc_adjoint_step");
    check(orc_adjoint_step(geom, s, Fu, F, sol, g, lam2, lam, gF, gs), "orc_adjoint_step");
    check_finite(lam, 27 * nw, "adjoint");
    check_finite(gF, 3 * nw, "dJ/dF");
    check_finite(gs, 10, "dJ/ds");

    /* D3Q19 (19 planes) */
    check(orc19_init(geom, rho0, u0, f), "orc19_init");
    check(orc19_step(geom, s, Fu, F, sol, f, g), "orc19_step");
    check(orc19_macro(geom, Fu, F, sol, g, rho, u), "orc19_macro");
    check_finite(g, 19 * nw, "d3q19 state");
    check(orc19_step_ex(geom, s, Fu, F, sol, wall_u, g, f), "orc19_step_ex");
    check_finite(f, 19 * nw, "d3q19 state, moving walls");

    free(rho0), free(u0), free(Ff), free(ut), free(solid), free(f), free(g), free(lam), free(lam2);
    free(rho), free(u), free(gF);
}

int main(void)
{
    const int cases[][12] = {
        {5, 4, 3, 1, 1, 0, 0, 0, 0, 5, 4, 3},   /* walls in x and y */
        {3, 5, 4, 1, 1, 1, 0, 0, 0, 3, 5, 4},   /* walled box */
        {1, 1, 6, 0, 0, 0, 0, 0, 0, 1, 1, 6},   /* thin periodic column */
        {2, 3, 1, 0, 1, 0, 0, 0, 0, 2, 3, 1},   /* one plane */
        {9, 8, 7, 0, 1, 0, 6, 2, 5, 4, 5, 4},   /* window wrapping the periodic axes */
    };
    for (unsigned c = 0; c < sizeof(cases) / sizeof(cases[0]); ++c)
        for (int solids = 0; solids < 2; ++solids)
            for (int field = 0; field < 2; ++field) run_case(cases[c], solids, field);
    if (failures) {
        fprintf(stderr, "%d failures\n", failures);
        return 1;
    }
    printf("oracle sanitizer run: ok\n");
    return 0;
}

/*
 * Plain FP64 CPU oracle of the D3Q27 cascaded lattice Boltzmann method with the
 * simplified central-moment set and the consistent forcing scheme of
 * Fei, Luo & Li, "Three-dimensional cascaded lattice Boltzmann method: improved
 * implementation and consistent forcing scheme", arXiv:1801.04586.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only tests/, the smoke check and the CPU-baseline leg of the
 * benchmark use it.  It shares no code, header, table or helper with the HIP
 * library.
 *
 * It is deliberately slow and literal.  Every matrix is dense 27x27 and is built
 * entrywise from its definition in the paper; the time step follows Steps 1-4
 * of Sec. II B in the paper's order.  No per-axis factorisation, fusion or
 * reordering is used.  Arithmetic is IEEE double throughout.
 *
 * Readings of the paper taken here (each is also pinned by a test):
 *  - Eq. (2): the z factor of the central moment is (e_iz - u_z)^p.
 *  - Eq. (12): slot 9 of the moment set is k_002 (printed twice as k_020);
 *    with this reading M built from the definition equals the printed Eq. (14).
 *  - Eq. (13): s_nu and s_2 are the same rate.
 *  - Eq. (16): the printed vector C is used as the forcing term.
 *  - F is a force density (Eq. (6) divides it by rho, Eq. (9) adds F/2).
 *  - Half-way bounce-back (Sec. III, not printed): a population leaving fluid
 *    node x towards a wall or a solid node returns to x reversed one step later,
 *    f_opp(i)(x, t+1) = f*_i(x, t).  Solid nodes are neither collided nor
 *    streamed; their populations are left as they are.
 *  - The velocity entering N(u) and N^-1 is the one of Eq. (9) evaluated from
 *    the pre-collision populations and the current force.
 *  - N^-1(u) is evaluated as N(-u): shifting the moments by +u and then by -u
 *    is the identity (binomial theorem); tests check N(u) N(-u) = I.
 *
 * Adjoint (not in the paper): the exact transpose of the discrete step above,
 * built from dense Jacobians by the chain rule; see orc_adjoint_step.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 27

/* ---- Eq. (1): discrete velocities, population order of the paper ---------- */
static const int EX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1,
                          0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1};
static const int EY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0,
                          1, -1, 1, -1, 1, 1, -1, -1, 1, 1, -1, -1};
static const int EZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1,
                          1, 1, -1, -1, 1, 1, 1, 1, -1, -1, -1, -1};

/* ---- Eq. (12): exponents (m, n, p) of the moment set (slot 9 = k_002) ----- */
static const int PX[Q] = {0, 1, 0, 0, 1, 1, 0, 2, 0, 0, 1, 1, 2, 2, 0, 0, 1, 2, 2, 0, 2, 1, 1, 1, 2, 2, 2};
static const int PY[Q] = {0, 0, 1, 0, 1, 0, 1, 0, 2, 0, 2, 0, 1, 0, 1, 2, 1, 2, 0, 2, 1, 2, 1, 2, 1, 2, 2};
static const int PZ[Q] = {0, 0, 0, 1, 0, 1, 1, 0, 0, 2, 0, 2, 0, 1, 2, 1, 1, 0, 2, 2, 1, 1, 2, 2, 2, 1, 2};

static const double CS2 = 1.0 / 3.0; /* c_s^2, Sec. II A */

static int e_of(int i, int axis) { return axis == 0 ? EX[i] : (axis == 1 ? EY[i] : EZ[i]); }
static int p_of(int a, int axis) { return axis == 0 ? PX[a] : (axis == 1 ? PY[a] : PZ[a]); }

/* x^n for the small exponents n = 0, 1, 2 (and 3 for derivatives) used here; x^0 = 1. */
static double ipow(double x, int n)
{
    switch (n) {
    case 0: return 1.0;
    case 1: return x;
    case 2: return x * x;
    default: {
        double r = 1.0;
        for (int k = 0; k < n; ++k) r *= x;
        return r;
    }
    }
}

/* binomial coefficient C(n, k) for 0 <= k <= n <= 2 */
static double binom(int n, int k)
{
    static const double tab[3][3] = {{1, 0, 0}, {1, 1, 0}, {1, 2, 1}};
    return tab[n][k];
}

/* opposite population: the index j with e_j = -e_i */
static int opposite(int i)
{
    for (int j = 0; j < Q; ++j)
        if (EX[j] == -EX[i] && EY[j] == -EY[i] && EZ[j] == -EZ[i]) return j;
    return -1;
}

/* ---- dense 27x27 helpers (row-major, A[r*Q + c]) ------------------------ */
static void matvec(const double *A, const double *x, double *y)
{
    for (int r = 0; r < Q; ++r) {
        double acc = 0.0;
        for (int c = 0; c < Q; ++c) acc += A[r * Q + c] * x[c];
        y[r] = acc;
    }
}

static void matTvec(const double *A, const double *x, double *y)
{
    for (int c = 0; c < Q; ++c) {
        double acc = 0.0;
        for (int r = 0; r < Q; ++r) acc += A[r * Q + c] * x[r];
        y[c] = acc;
    }
}

/* Gauss-Jordan elimination with partial pivoting; returns 0 on success. */
static int invert(int n, const double *A, double *Ainv)
{
    double *W = (double *)malloc(sizeof(double) * (size_t)n * 2 * n);
    if (!W) return 2;
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < 2 * n; ++c)
            W[r * 2 * n + c] = c < n ? A[r * n + c] : (c - n == r ? 1.0 : 0.0);
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (fabs(W[r * 2 * n + col]) > fabs(W[piv * 2 * n + col])) piv = r;
        if (fabs(W[piv * 2 * n + col]) < 1e-300) { free(W); return 1; }
        if (piv != col)
            for (int c = 0; c < 2 * n; ++c) {
                double t = W[col * 2 * n + c];
                W[col * 2 * n + c] = W[piv * 2 * n + c];
                W[piv * 2 * n + c] = t;
            }
        double d = W[col * 2 * n + col];
        for (int c = 0; c < 2 * n; ++c) W[col * 2 * n + c] /= d;
        for (int r = 0; r < n; ++r) {
            if (r == col) continue;
            double m = W[r * 2 * n + col];
            if (m == 0.0) continue;
            for (int c = 0; c < 2 * n; ++c) W[r * 2 * n + c] -= m * W[col * 2 * n + c];
        }
    }
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) Ainv[r * n + c] = W[r * 2 * n + n + c];
    free(W);
    return 0;
}

/* ======================================================================== */
/* Matrices of Sec. II                                                       */
/* ======================================================================== */

/* Eq. (2) + Eq. (4): K(u) = N(u) M, entry (a, i) = prod_alpha (e_i,alpha - u_alpha)^p_a,alpha.
 * With u = 0 this is the raw-moment matrix M of Eq. (14). */
void orc_matrix_K(const double *u, double *K)
{
    double pw[Q][3][3]; /* pw[i][axis][p] = (e_i,axis - u_axis)^p */
    for (int i = 0; i < Q; ++i)
        for (int ax = 0; ax < 3; ++ax)
            for (int p = 0; p < 3; ++p) pw[i][ax][p] = ipow((double)e_of(i, ax) - u[ax], p);
    for (int a = 0; a < Q; ++a)
        for (int i = 0; i < Q; ++i) K[a * Q + i] = pw[i][0][PX[a]] * pw[i][1][PY[a]] * pw[i][2][PZ[a]];
}

/* Eq. (4) + Eq. (14): M, the raw moments k_mnp = <f | e_x^m e_y^n e_z^p>. */
void orc_matrix_M(double *M)
{
    const double zero[3] = {0.0, 0.0, 0.0};
    orc_matrix_K(zero, M);
}

/* Eq. (4): shift matrix N(u) from the binomial expansion of (e - u)^p, so that
 * central moment a = sum_b N_ab raw moment b (example row N_4 in Sec. II B). */
void orc_matrix_N(const double *u, double *N)
{
    for (int a = 0; a < Q; ++a)
        for (int b = 0; b < Q; ++b) {
            double v = 1.0;
            for (int ax = 0; ax < 3; ++ax) {
                int pa = p_of(a, ax), pb = p_of(b, ax);
                if (pb > pa) { v = 0.0; break; }
                v *= binom(pa, pb) * ipow(-u[ax], pa - pb);
            }
            N[a * Q + b] = v;
        }
}

/* Eq. (7): N^-1(u), evaluated as N(-u) (a shift by -u undoes a shift by +u). */
void orc_matrix_Ninv(const double *u, double *Ninv)
{
    const double mu[3] = {-u[0], -u[1], -u[2]};
    orc_matrix_N(mu, Ninv);
}

/* Eq. (14) inverse, by Gauss-Jordan elimination of the matrix from the definition. */
int orc_matrix_Minv(double *Minv)
{
    double M[Q * Q];
    orc_matrix_M(M);
    return invert(Q, M, Minv);
}

/* Generic dense inverse, exposed for tests (n <= 64). */
int orc_invert(int n, const double *A, double *Ainv) { return invert(n, A, Ainv); }

/* Eq. (13): block-diagonal relaxation matrix.  s[] = {s0, s1, s2 (= s_nu), s2b,
 * s3, s3b, s4, s4b, s5, s6}; s_+ = (s2b + 2 s2)/3, s_- = (s2b - s2)/3.  S is
 * linear in the ten rates. */
void orc_matrix_S(const double *s, double *S)
{
    const double s0 = s[0], s1 = s[1], s2 = s[2], s2b = s[3], s3 = s[4], s3b = s[5];
    const double s4 = s[6], s4b = s[7], s5 = s[8], s6 = s[9];
    const double sp = (s2b + 2.0 * s2) / 3.0, sm = (s2b - s2) / 3.0;
    double diag[Q] = {s0, s1, s1, s1, s2, s2, s2, 0, 0, 0, s3, s3, s3, s3, s3, s3, s3b,
                      s4, s4, s4, s4b, s4b, s4b, s5, s5, s5, s6};
    memset(S, 0, sizeof(double) * Q * Q);
    for (int a = 0; a < Q; ++a) S[a * Q + a] = diag[a];
    for (int r = 7; r <= 9; ++r)
        for (int c = 7; c <= 9; ++c) S[r * Q + c] = (r == c) ? sp : sm;
}

/* Eq. (15): central-moment equilibria of the continuous Maxwellian. */
void orc_teq(double rho, double *teq)
{
    memset(teq, 0, sizeof(double) * Q);
    teq[0] = rho;
    teq[7] = teq[8] = teq[9] = rho * CS2;
    teq[17] = teq[18] = teq[19] = rho * CS2 * CS2;
    teq[26] = rho * CS2 * CS2 * CS2;
}

/* Eq. (16), as printed: forcing terms in central-moment space. */
void orc_cvec(const double *F, double *C)
{
    const double Fx = F[0], Fy = F[1], Fz = F[2];
    memset(C, 0, sizeof(double) * Q);
    C[1] = Fx;
    C[2] = Fy;
    C[3] = Fz;
    C[10] = Fx * CS2;
    C[11] = Fx * CS2;
    C[12] = Fy * CS2;
    C[13] = Fz * CS2;
    C[14] = Fy * CS2;
    C[15] = Fz * CS2;
    C[23] = Fx * CS2 * CS2;
    C[24] = Fy * CS2 * CS2;
    C[25] = Fz * CS2 * CS2;
}

void orc_velocities(int *e)
{
    for (int i = 0; i < Q; ++i) {
        e[3 * i] = EX[i];
        e[3 * i + 1] = EY[i];
        e[3 * i + 2] = EZ[i];
    }
}

void orc_exponents(int *p)
{
    for (int a = 0; a < Q; ++a) {
        p[3 * a] = PX[a];
        p[3 * a + 1] = PY[a];
        p[3 * a + 2] = PZ[a];
    }
}

/* ======================================================================== */
/* One node: Eq. (9), Steps 1-3                                             */
/* ======================================================================== */

/* Eq. (9): rho = sum f, rho u = sum f e + F/2. */
static void macro_node(const double *f, const double *F, double *rho, double *u)
{
    double r = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
    for (int i = 0; i < Q; ++i) {
        r += f[i];
        jx += f[i] * EX[i];
        jy += f[i] * EY[i];
        jz += f[i] * EZ[i];
    }
    *rho = r;
    u[0] = (jx + 0.5 * F[0]) / r;
    u[1] = (jy + 0.5 * F[1]) / r;
    u[2] = (jz + 0.5 * F[2]) / r;
}

typedef struct {
    double S[Q * Q];
    double Minv[Q * Q];
} orc_consts;

static int consts_init(orc_consts *k, const double *s)
{
    orc_matrix_S(s, k->S);
    return orc_matrix_Minv(k->Minv);
}

/* Steps 1-3 of Sec. II B for one node: central moments by the definition
 * Eq. (2), collision Eq. (5), reconstruction Eq. (7) via N^-1 then M^-1. */
static void collide_node(const orc_consts *k, const double *f, const double *F, double *fs)
{
    double rho, u[3], K[Q * Q], Ninv[Q * Q];
    double T[Q], Tt[Q], teq[Q], C[Q], SA[Q], SB[Q], SC[Q], Ts[Q];
    macro_node(f, F, &rho, u);
    orc_matrix_K(u, K);      /* Step 1 */
    matvec(K, f, Tt);
    orc_teq(rho, teq);       /* Step 2 */
    orc_cvec(F, C);
    matvec(k->S, Tt, SA);
    matvec(k->S, teq, SB);
    matvec(k->S, C, SC);
    for (int a = 0; a < Q; ++a) Ts[a] = Tt[a] - SA[a] + SB[a] + C[a] - 0.5 * SC[a];
    orc_matrix_Ninv(u, Ninv); /* Step 3 */
    matvec(Ninv, Ts, T);
    matvec(k->Minv, T, fs);
}

/* Single-node collision exposed for tests: f (27) -> f* (27). */
int orc_collide(const double *f, const double *F, const double *s, double *fs)
{
    orc_consts k;
    if (consts_init(&k, s)) return 1;
    collide_node(&k, f, F, fs);
    return 0;
}

/* Generalised local equilibrium (Sec. II B): f_eq = (N M)^-1 T_eq = M^-1 N(-u) T_eq(rho). */
int orc_equilibrium(double rho, const double *u, double *feq)
{
    double Minv[Q * Q], Ninv[Q * Q], teq[Q], T[Q];
    if (orc_matrix_Minv(Minv)) return 1;
    orc_teq(rho, teq);
    orc_matrix_Ninv(u, Ninv);
    matvec(Ninv, teq, T);
    matvec(Minv, T, feq);
    return 0;
}

/* ======================================================================== */
/* Lattice: geometry, windows, streaming (Eq. (8)) with half-way bounce-back */
/* ======================================================================== */
/*
 * geom[12] = {gx, gy, gz, wall_x, wall_y, wall_z, ox, oy, oz, wx, wy, wz}.
 * The lattice is gx*gy*gz nodes; axis a is periodic when wall_a == 0 and has
 * half-way bounce-back walls at both ends when wall_a == 1.  Arrays hold the
 * window [ox, ox+wx) x [oy, oy+wy) x [oz, oz+wz) (global coordinates, wrapped
 * on periodic axes); the whole lattice is the window with origin 0 and
 * w = g.  Node id n = x + wx*(y + wy*z), populations as [27][n].  Streaming
 * targets outside a partial window are dropped (their destinations become
 * NaN), so after k steps every node at least k nodes inside the window edge
 * of a partial axis is exact.
 */
typedef struct {
    int g[3], wall[3], o[3], w[3];
    long n;
} orc_geom;

static int geom_read(const int *gi, orc_geom *G)
{
    for (int a = 0; a < 3; ++a) {
        G->g[a] = gi[a];
        G->wall[a] = gi[3 + a];
        G->o[a] = gi[6 + a];
        G->w[a] = gi[9 + a];
        if (G->g[a] < 1 || G->w[a] < 1 || G->w[a] > G->g[a]) return 1;
        if (G->wall[a] && (G->o[a] < 0 || G->o[a] + G->w[a] > G->g[a])) return 1;
    }
    G->n = (long)G->w[0] * G->w[1] * G->w[2];
    return 0;
}

static int imod(int a, int m)
{
    int r = a % m;
    return r < 0 ? r + m : r;
}

/* Window-local coordinate of global neighbour coordinate c (unwrapped) on axis a.
 * Returns -1 if c is beyond a wall, -2 if outside a partial window, else index. */
static int locate(const orc_geom *G, int a, int c)
{
    if (G->wall[a] && (c < 0 || c >= G->g[a])) return -1;
    int cg = imod(c, G->g[a]);
    int l = imod(cg - G->o[a], G->g[a]);
    return l < G->w[a] ? l : -2;
}

static void force_at(const double *Fu, const double *Ff, long n, long node, double *F)
{
    for (int a = 0; a < 3; ++a) F[a] = (Fu ? Fu[a] : 0.0) + (Ff ? Ff[a * n + node] : 0.0);
}

/*
 * One time step (Steps 1-4): collide every fluid node, then stream with
 * half-way bounce-back.  fin/fout: [27][n] pre-collision populations at t and
 * t+1.  Fu: uniform force (3) or NULL; Ff: per-node force [3][n] or NULL (the
 * force at a node is Fu + Ff).  solid: [n] (1 = solid) or NULL.
 */
int orc_step(const int *geom, const double *s, const double *Fu, const double *Ff,
             const uint8_t *solid, const double *fin, double *fout)
{
    orc_geom G;
    orc_consts k;
    if (geom_read(geom, &G)) return 1;
    if (consts_init(&k, s)) return 2;
    const long n = G.n;
    const double nan = NAN;
    for (long idx = 0; idx < (long)Q * n; ++idx) fout[idx] = nan;
    /* solid nodes keep their populations */
    if (solid)
        for (long node = 0; node < n; ++node)
            if (solid[node])
                for (int i = 0; i < Q; ++i) fout[(long)i * n + node] = fin[(long)i * n + node];
    int opp[Q];
    for (int i = 0; i < Q; ++i) opp[i] = opposite(i);

#pragma omp parallel for schedule(static)
    for (long node = 0; node < n; ++node) {
        if (solid && solid[node]) continue;
        const int x = (int)(node % G.w[0]);
        const int y = (int)((node / G.w[0]) % G.w[1]);
        const int z = (int)(node / ((long)G.w[0] * G.w[1]));
        double f[Q], fs[Q], F[3];
        for (int i = 0; i < Q; ++i) f[i] = fin[(long)i * n + node];
        force_at(Fu, Ff, n, node, F);
        collide_node(&k, f, F, fs);
        for (int i = 0; i < Q; ++i) {
            /* Eq. (8): f_i(x + e_i, t+1) = f*_i(x, t) */
            const int lx = locate(&G, 0, G.o[0] + x + EX[i]);
            const int ly = locate(&G, 1, G.o[1] + y + EY[i]);
            const int lz = locate(&G, 2, G.o[2] + z + EZ[i]);
            if (lx == -2 || ly == -2 || lz == -2) continue; /* leaves a partial window */
            long tgt = -1;
            if (lx >= 0 && ly >= 0 && lz >= 0) {
                tgt = (long)lx + (long)G.w[0] * ((long)ly + (long)G.w[1] * lz);
                if (solid && solid[tgt]) tgt = -1;
            }
            if (tgt >= 0)
                fout[(long)i * n + tgt] = fs[i];
            else /* half-way bounce-back: back to x, reversed */
                fout[(long)opp[i] * n + node] = fs[i];
        }
    }
    return 0;
}

/* Eq. (9) on every node: rho [n], u [3][n]; solid nodes get rho = u = 0. */
int orc_macro(const int *geom, const double *Fu, const double *Ff, const uint8_t *solid,
              const double *f, double *rho, double *u)
{
    orc_geom G;
    if (geom_read(geom, &G)) return 1;
    const long n = G.n;
#pragma omp parallel for schedule(static)
    for (long node = 0; node < n; ++node) {
        if (solid && solid[node]) {
            rho[node] = 0.0;
            u[node] = u[n + node] = u[2 * n + node] = 0.0;
            continue;
        }
        double fl[Q], F[3], r, uu[3];
        for (int i = 0; i < Q; ++i) fl[i] = f[(long)i * n + node];
        force_at(Fu, Ff, n, node, F);
        macro_node(fl, F, &r, uu);
        rho[node] = r;
        u[node] = uu[0];
        u[n + node] = uu[1];
        u[2 * n + node] = uu[2];
    }
    return 0;
}

/* Initial state: f = f_eq(rho0(x), u0(x)) at every node (solids included). */
int orc_init(const int *geom, const double *rho0, const double *u0, double *f)
{
    orc_geom G;
    double Minv[Q * Q];
    if (geom_read(geom, &G)) return 1;
    if (orc_matrix_Minv(Minv)) return 2;
    const long n = G.n;
#pragma omp parallel for schedule(static)
    for (long node = 0; node < n; ++node) {
        double u[3], Ninv[Q * Q], teq[Q], T[Q], fe[Q];
        const double r = rho0 ? rho0[node] : 1.0;
        for (int a = 0; a < 3; ++a) u[a] = u0 ? u0[(long)a * n + node] : 0.0;
        orc_teq(r, teq);
        orc_matrix_Ninv(u, Ninv);
        matvec(Ninv, teq, T);
        matvec(Minv, T, fe);
        for (int i = 0; i < Q; ++i) f[(long)i * n + node] = fe[i];
    }
    return 0;
}

/* ======================================================================== */
/* Adjoint of the discrete step (exact transpose, dense Jacobians)           */
/* ======================================================================== */
/*
 * Per node the step is f* = Phi(f, F, s) with
 *   rho = 1^T f, u = (E^T f + F/2)/rho, K = K(u) (Eq. (2)), L = K^-1 = M^-1 N(-u),
 *   Tt = K f, Ts = Tt - S (Tt - rho Ehat) + (I - S/2) C(F), f* = L Ts,
 * where Ehat = T_eq/rho (Eq. (15)) and C is linear in F (Eq. (16)).  Writing
 * dK_a = dK/du_a and using dL/du_a = -L dK_a L:
 *   g_a   = dL/du_a Ts + L (I - S) dK_a f = L [ (I - S) dK_a f - dK_a f* ]
 *   d(f*)/df = L (I - S) K + L S Ehat 1^T + sum_a g_a (e_a - u_a 1)^T / rho
 *   d(f*)/dF_a = L (I - S/2) dC/dF_a + g_a / (2 rho)
 *   d(f*)/ds_k = L (dS/ds_k) (rho Ehat - Tt - C/2),  dS/ds_k = S(unit_k)
 * The step's streaming with bounce-back is a permutation P, so the adjoint of
 * f(t+1) = P Phi(f(t)) is lambda(t) = (dPhi/df)^T P^T lambda(t+1), where
 * (P^T lambda)_i(x) = lambda_i(x + e_i) for a fluid target and lambda_opp(i)(x)
 * for a bounced link.
 */

/* dK/du_axis, entry (a, i) = -p_a,axis (e_i,axis - u_axis)^(p-1) prod_{b != axis} (...) */
static void matrix_dK(const double *u, int axis, double *dK)
{
    for (int a = 0; a < Q; ++a)
        for (int i = 0; i < Q; ++i) {
            double v = 1.0;
            for (int ax = 0; ax < 3; ++ax) {
                const int p = p_of(a, ax);
                const double d = (double)e_of(i, ax) - u[ax];
                if (ax == axis)
                    v *= (p == 0) ? 0.0 : -(double)p * ipow(d, p - 1);
                else
                    v *= ipow(d, p);
            }
            dK[a * Q + i] = v;
        }
}

/*
 * Per-node adjoint: given pre-collision f, force F and incoming adjoint a =
 * dJ/d(f*) (27), return lam = (d(f*)/df)^T a, and add (d(f*)/dF)^T a to gF[3]
 * and (d(f*)/ds)^T a to gs[10].
 */
static void adjoint_node(const double *s, const double *S, const double *f, const double *F,
                         const double *a, double *lam, double *gF, double *gs)
{
    double rho, u[3], K[Q * Q], L[Q * Q], Tt[Q], teq[Q], C[Q], Ts[Q], fs[Q];
    double SA[Q], SB[Q], SC[Q];
    macro_node(f, F, &rho, u);
    orc_matrix_K(u, K);
    if (invert(Q, K, L)) { for (int i = 0; i < Q; ++i) lam[i] = NAN; return; }
    matvec(K, f, Tt);
    orc_teq(rho, teq);
    orc_cvec(F, C);
    matvec(S, Tt, SA);
    matvec(S, teq, SB);
    matvec(S, C, SC);
    for (int b = 0; b < Q; ++b) Ts[b] = Tt[b] - SA[b] + SB[b] + C[b] - 0.5 * SC[b];
    matvec(L, Ts, fs);

    double La[Q]; /* L^T a */
    matTvec(L, a, La);

    /* term 1: K^T (I - S)^T L^T a */
    double IS_La[Q], t1[Q];
    matTvec(S, La, IS_La);
    for (int b = 0; b < Q; ++b) IS_La[b] = La[b] - IS_La[b];
    matTvec(K, IS_La, t1);
    /* term 2: 1 * (Ehat^T S^T L^T a) */
    double SLa[Q], ehat[Q], t2 = 0.0;
    matTvec(S, La, SLa);
    orc_teq(1.0, ehat);
    for (int b = 0; b < Q; ++b) t2 += ehat[b] * SLa[b];
    /* terms with g_a */
    double ga_dot[3];
    for (int ax = 0; ax < 3; ++ax) {
        double dK[Q * Q], v1[Q], v2[Q], Sv1[Q], w[Q], g[Q];
        matrix_dK(u, ax, dK);
        matvec(dK, f, v1);
        matvec(S, v1, Sv1);
        matvec(dK, fs, v2);
        for (int b = 0; b < Q; ++b) w[b] = v1[b] - Sv1[b] - v2[b];
        matvec(L, w, g);
        double d = 0.0;
        for (int i = 0; i < Q; ++i) d += g[i] * a[i];
        ga_dot[ax] = d;
    }
    for (int i = 0; i < Q; ++i) {
        double v = t1[i] + t2;
        v += ga_dot[0] * ((double)EX[i] - u[0]) / rho;
        v += ga_dot[1] * ((double)EY[i] - u[1]) / rho;
        v += ga_dot[2] * ((double)EZ[i] - u[2]) / rho;
        lam[i] = v;
    }
    /* force: L (I - S/2) dC/dF_a + g_a/(2 rho) */
    for (int ax = 0; ax < 3; ++ax) {
        double unit[3] = {0.0, 0.0, 0.0}, dC[Q], SdC[Q], v[Q], Lv[Q];
        unit[ax] = 1.0;
        orc_cvec(unit, dC);
        matvec(S, dC, SdC);
        for (int b = 0; b < Q; ++b) v[b] = dC[b] - 0.5 * SdC[b];
        matvec(L, v, Lv);
        double d = 0.0;
        for (int i = 0; i < Q; ++i) d += Lv[i] * a[i];
        gF[ax] += d + ga_dot[ax] / (2.0 * rho);
    }
    /* rates: L S(unit_k) (rho Ehat - Tt - C/2) */
    double r[Q];
    for (int b = 0; b < Q; ++b) r[b] = teq[b] - Tt[b] - 0.5 * C[b];
    for (int kk = 0; kk < 10; ++kk) {
        double unit[10] = {0}, Sk[Q * Q], v[Q], Lv[Q];
        unit[kk] = 1.0;
        orc_matrix_S(unit, Sk);
        matvec(Sk, r, v);
        matvec(L, v, Lv);
        double d = 0.0;
        for (int i = 0; i < Q; ++i) d += Lv[i] * a[i];
        gs[kk] += d;
    }
    (void)s;
}

/*
 * One adjoint step.  f_t: pre-collision populations at t ([27][n]);
 * lam_next: dJ/df(t+1) ([27][n]); lam_out: dJ/df(t) ([27][n]);
 * gF: [3][n] accumulated dJ/dF; gs: [10] accumulated dJ/ds.
 * Solid nodes: lam_out = lam_next (their populations are carried unchanged).
 * Gathers from outside a partial window give NaN.
 */
int orc_adjoint_step(const int *geom, const double *s, const double *Fu, const double *Ff,
                     const uint8_t *solid, const double *f_t, const double *lam_next,
                     double *lam_out, double *gF, double *gs)
{
    orc_geom G;
    double S[Q * Q];
    if (geom_read(geom, &G)) return 1;
    orc_matrix_S(s, S);
    const long n = G.n;
    int opp[Q];
    for (int i = 0; i < Q; ++i) opp[i] = opposite(i);
    double gs_tot[10] = {0};

#pragma omp parallel
    {
        double gs_loc[10] = {0};
#pragma omp for schedule(static)
        for (long node = 0; node < n; ++node) {
            if (solid && solid[node]) {
                for (int i = 0; i < Q; ++i) lam_out[(long)i * n + node] = lam_next[(long)i * n + node];
                continue;
            }
            const int x = (int)(node % G.w[0]);
            const int y = (int)((node / G.w[0]) % G.w[1]);
            const int z = (int)(node / ((long)G.w[0] * G.w[1]));
            double f[Q], F[3], a[Q], lam[Q], gF_loc[3] = {0, 0, 0};
            for (int i = 0; i < Q; ++i) f[i] = f_t[(long)i * n + node];
            force_at(Fu, Ff, n, node, F);
            for (int i = 0; i < Q; ++i) { /* a = (P^T lambda(t+1))(x) */
                const int lx = locate(&G, 0, G.o[0] + x + EX[i]);
                const int ly = locate(&G, 1, G.o[1] + y + EY[i]);
                const int lz = locate(&G, 2, G.o[2] + z + EZ[i]);
                if (lx == -2 || ly == -2 || lz == -2) { a[i] = NAN; continue; }
                long tgt = -1;
                if (lx >= 0 && ly >= 0 && lz >= 0) {
                    tgt = (long)lx + (long)G.w[0] * ((long)ly + (long)G.w[1] * lz);
                    if (solid && solid[tgt]) tgt = -1;
                }
                a[i] = tgt >= 0 ? lam_next[(long)i * n + tgt] : lam_next[(long)opp[i] * n + node];
            }
            adjoint_node(s, S, f, F, a, lam, gF_loc, gs_loc);
            for (int i = 0; i < Q; ++i) lam_out[(long)i * n + node] = lam[i];
            if (gF)
                for (int ax = 0; ax < 3; ++ax) gF[(long)ax * n + node] += gF_loc[ax];
        }
#pragma omp critical
        for (int kk = 0; kk < 10; ++kk) gs_tot[kk] += gs_loc[kk];
    }
    if (gs)
        for (int kk = 0; kk < 10; ++kk) gs[kk] += gs_tot[kk];
    return 0;
}

/*
 * Loss J = 1/2 sum over fluid nodes |u(x) - u_target(x)|^2 with u from Eq. (9)
 * on the populations f.  Writes lam = dJ/df ([27][n], zero on solids), adds the
 * direct dJ/dF (u depends on F/2) to gF ([3][n]) and returns J in *J.
 */
int orc_loss_seed(const int *geom, const double *Fu, const double *Ff, const uint8_t *solid,
                  const double *f, const double *u_target, double *lam, double *gF, double *J)
{
    orc_geom G;
    if (geom_read(geom, &G)) return 1;
    const long n = G.n;
    double Jt = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : Jt)
    for (long node = 0; node < n; ++node) {
        if (solid && solid[node]) {
            for (int i = 0; i < Q; ++i) lam[(long)i * n + node] = 0.0;
            continue;
        }
        double fl[Q], F[3], rho, u[3], d[3];
        for (int i = 0; i < Q; ++i) fl[i] = f[(long)i * n + node];
        force_at(Fu, Ff, n, node, F);
        macro_node(fl, F, &rho, u);
        for (int ax = 0; ax < 3; ++ax) d[ax] = u[ax] - u_target[(long)ax * n + node];
        Jt += 0.5 * (d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        for (int i = 0; i < Q; ++i)
            lam[(long)i * n + node] = (d[0] * ((double)EX[i] - u[0]) + d[1] * ((double)EY[i] - u[1]) +
                                       d[2] * ((double)EZ[i] - u[2])) / rho;
        if (gF)
            for (int ax = 0; ax < 3; ++ax) gF[(long)ax * n + node] += d[ax] / (2.0 * rho);
    }
    *J = Jt;
    return 0;
}

int orc_abi_version(void) { return 1; }

/* Threads the OpenMP loops above use. */
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads for the following parallel loops (n >= 1); no effect without OpenMP. */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ======================================================================== */
/* D3Q19 cascaded LBM of Appendix A                                          */
/* ======================================================================== */
/*
 * The same scheme on the D3Q19 lattice: velocities of Eq. (A1), the 19 central
 * moments of Eq. (A2) (its slot 9, printed as k~_020 a second time, read as
 * k~_002 as for Eq. (12); M from the definition then equals the printed
 * Eq. (A4), which a test checks), the block relaxation of Eq. (A3) with s3 for
 * the six third-order moments and s4 for the three fourth-order ones, the
 * equilibria of Eq. (A5) and the forcing terms of Eq. (A6).  Matrices are dense
 * 19x19 and built entrywise; the step is Steps 1-4 of Sec. II B; streaming and
 * bounce-back are those of the D3Q27 oracle above.  Rate array as above:
 * {s0, s1, s2, s2b, s3, s3b, s4, s4b, s5, s6}; s3b, s4b, s5, s6 have no moment
 * here and are ignored.
 */
#define Q19 19

/* Eq. (A1) */
static const int EX19[Q19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static const int EY19[Q19] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1};
static const int EZ19[Q19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1};

/* Eq. (A2): k000, k100, k010, k001, k110, k101, k011, k200, k020, k002, k120, k102,
 * k210, k201, k012, k021, k220, k202, k022 */
static const int PX19[Q19] = {0, 1, 0, 0, 1, 1, 0, 2, 0, 0, 1, 1, 2, 2, 0, 0, 2, 2, 0};
static const int PY19[Q19] = {0, 0, 1, 0, 1, 0, 1, 0, 2, 0, 2, 0, 1, 0, 1, 2, 2, 0, 2};
static const int PZ19[Q19] = {0, 0, 0, 1, 0, 1, 1, 0, 0, 2, 0, 2, 0, 1, 2, 1, 0, 2, 2};

static int e19(int i, int axis) { return axis == 0 ? EX19[i] : (axis == 1 ? EY19[i] : EZ19[i]); }
static int p19(int a, int axis) { return axis == 0 ? PX19[a] : (axis == 1 ? PY19[a] : PZ19[a]); }

static void matvec19(const double *A, const double *x, double *y)
{
    for (int r = 0; r < Q19; ++r) {
        double acc = 0.0;
        for (int c = 0; c < Q19; ++c) acc += A[r * Q19 + c] * x[c];
        y[r] = acc;
    }
}

static int opposite19(int i)
{
    for (int j = 0; j < Q19; ++j)
        if (EX19[j] == -EX19[i] && EY19[j] == -EY19[i] && EZ19[j] == -EZ19[i]) return j;
    return -1;
}

/* Eq. (2) on D3Q19: K(u) = N(u) M, entry (a, i) = prod_alpha (e_i,alpha - u_alpha)^p_a,alpha */
void orc19_matrix_K(const double *u, double *K)
{
    for (int a = 0; a < Q19; ++a)
        for (int i = 0; i < Q19; ++i) {
            double v = 1.0;
            for (int ax = 0; ax < 3; ++ax) v *= ipow((double)e19(i, ax) - u[ax], p19(a, ax));
            K[a * Q19 + i] = v;
        }
}

/* Eq. (A4): raw moments k_mnp = <f | e_x^m e_y^n e_z^p> */
void orc19_matrix_M(double *M)
{
    const double zero[3] = {0.0, 0.0, 0.0};
    orc19_matrix_K(zero, M);
}

/* Shift matrix N(u) of the D3Q19 set, from the binomial expansion of (e - u)^p
 * (every raw moment it needs is in the set: the set is closed under lowering
 * exponents). */
void orc19_matrix_N(const double *u, double *N)
{
    for (int a = 0; a < Q19; ++a)
        for (int b = 0; b < Q19; ++b) {
            double v = 1.0;
            for (int ax = 0; ax < 3; ++ax) {
                int pa = p19(a, ax), pb = p19(b, ax);
                if (pb > pa) { v = 0.0; break; }
                v *= binom(pa, pb) * ipow(-u[ax], pa - pb);
            }
            N[a * Q19 + b] = v;
        }
}

int orc19_matrix_Minv(double *Minv)
{
    double M[Q19 * Q19];
    orc19_matrix_M(M);
    return invert(Q19, M, Minv);
}

/* Eq. (A3) */
void orc19_matrix_S(const double *s, double *S)
{
    const double s0 = s[0], s1 = s[1], s2 = s[2], s2b = s[3], s3 = s[4], s4 = s[6];
    const double sp = (s2b + 2.0 * s2) / 3.0, sm = (s2b - s2) / 3.0;
    double diag[Q19] = {s0, s1, s1, s1, s2, s2, s2, 0, 0, 0, s3, s3, s3, s3, s3, s3, s4, s4, s4};
    memset(S, 0, sizeof(double) * Q19 * Q19);
    for (int a = 0; a < Q19; ++a) S[a * Q19 + a] = diag[a];
    for (int r = 7; r <= 9; ++r)
        for (int c = 7; c <= 9; ++c) S[r * Q19 + c] = (r == c) ? sp : sm;
}

/* Eq. (A5) */
void orc19_teq(double rho, double *teq)
{
    memset(teq, 0, sizeof(double) * Q19);
    teq[0] = rho;
    teq[7] = teq[8] = teq[9] = rho * CS2;
    teq[16] = teq[17] = teq[18] = rho * CS2 * CS2;
}

/* Eq. (A6) */
void orc19_cvec(const double *F, double *C)
{
    const double Fx = F[0], Fy = F[1], Fz = F[2];
    memset(C, 0, sizeof(double) * Q19);
    C[1] = Fx;
    C[2] = Fy;
    C[3] = Fz;
    C[10] = Fx * CS2;
    C[11] = Fx * CS2;
    C[12] = Fy * CS2;
    C[13] = Fz * CS2;
    C[14] = Fy * CS2;
    C[15] = Fz * CS2;
}

void orc19_velocities(int *e)
{
    for (int i = 0; i < Q19; ++i) {
        e[3 * i] = EX19[i];
        e[3 * i + 1] = EY19[i];
        e[3 * i + 2] = EZ19[i];
    }
}

void orc19_exponents(int *p)
{
    for (int a = 0; a < Q19; ++a) {
        p[3 * a] = PX19[a];
        p[3 * a + 1] = PY19[a];
        p[3 * a + 2] = PZ19[a];
    }
}

static void macro_node19(const double *f, const double *F, double *rho, double *u)
{
    double r = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
    for (int i = 0; i < Q19; ++i) {
        r += f[i];
        jx += f[i] * EX19[i];
        jy += f[i] * EY19[i];
        jz += f[i] * EZ19[i];
    }
    *rho = r;
    u[0] = (jx + 0.5 * F[0]) / r;
    u[1] = (jy + 0.5 * F[1]) / r;
    u[2] = (jz + 0.5 * F[2]) / r;
}

typedef struct {
    double S[Q19 * Q19];
    double Minv[Q19 * Q19];
} orc19_consts;

static int consts19_init(orc19_consts *k, const double *s)
{
    orc19_matrix_S(s, k->S);
    return orc19_matrix_Minv(k->Minv);
}

/* Steps 1-3 of Sec. II B on one D3Q19 node */
static void collide_node19(const orc19_consts *k, const double *f, const double *F, double *fs)
{
    double rho, u[3], K[Q19 * Q19], Ninv[Q19 * Q19];
    double T[Q19], Tt[Q19], teq[Q19], C[Q19], SA[Q19], SB[Q19], SC[Q19], Ts[Q19];
    macro_node19(f, F, &rho, u);
    orc19_matrix_K(u, K);
    matvec19(K, f, Tt);
    orc19_teq(rho, teq);
    orc19_cvec(F, C);
    matvec19(k->S, Tt, SA);
    matvec19(k->S, teq, SB);
    matvec19(k->S, C, SC);
    for (int a = 0; a < Q19; ++a) Ts[a] = Tt[a] - SA[a] + SB[a] + C[a] - 0.5 * SC[a];
    const double um[3] = {-u[0], -u[1], -u[2]}; /* N^-1(u) = N(-u) */
    orc19_matrix_N(um, Ninv);
    matvec19(Ninv, Ts, T);
    matvec19(k->Minv, T, fs);
}

int orc19_collide(const double *f, const double *F, const double *s, double *fs)
{
    orc19_consts k;
    if (consts19_init(&k, s)) return 1;
    collide_node19(&k, f, F, fs);
    return 0;
}

/* Generalised local equilibrium on D3Q19: f_eq = M^-1 N(-u) T_eq(rho) */
int orc19_equilibrium(double rho, const double *u, double *feq)
{
    double Minv[Q19 * Q19], Ninv[Q19 * Q19], teq[Q19], T[Q19];
    const double um[3] = {-u[0], -u[1], -u[2]};
    if (orc19_matrix_Minv(Minv)) return 1;
    orc19_teq(rho, teq);
    orc19_matrix_N(um, Ninv);
    matvec19(Ninv, teq, T);
    matvec19(Minv, T, feq);
    return 0;
}

/* D3Q19 rest-state weights (Appendix A): 1/3, 1/18, 1/36 by the number of nonzero components. */
static double weight19(int i)
{
    const int k = abs(EX19[i]) + abs(EY19[i]) + abs(EZ19[i]);
    return k == 0 ? 1.0 / 3.0 : (k == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
}

/* One D3Q19 time step; arguments as orc_step, populations [19][n].  wall_u: velocities of the
 * wall faces as for orc_step_ex (the D3Q27 MRT section below), or NULL for walls at rest; a link
 * leaving fluid node x through moving faces returns reversed with -2 w_i (e_i . u_w)/c_s^2,
 * u_w the mean velocity of the faces it crosses. */
int orc19_step_ex(const int *geom, const double *s, const double *Fu, const double *Ff,
                  const uint8_t *solid, const double *wall_u, const double *fin, double *fout)
{
    orc_geom G;
    orc19_consts k;
    if (geom_read(geom, &G)) return 1;
    if (consts19_init(&k, s)) return 2;
    const long n = G.n;
    for (long idx = 0; idx < (long)Q19 * n; ++idx) fout[idx] = NAN;
    if (solid)
        for (long node = 0; node < n; ++node)
            if (solid[node])
                for (int i = 0; i < Q19; ++i) fout[(long)i * n + node] = fin[(long)i * n + node];
    int opp[Q19];
    for (int i = 0; i < Q19; ++i) opp[i] = opposite19(i);

#pragma omp parallel for schedule(static)
    for (long node = 0; node < n; ++node) {
        if (solid && solid[node]) continue;
        const int x = (int)(node % G.w[0]);
        const int y = (int)((node / G.w[0]) % G.w[1]);
        const int z = (int)(node / ((long)G.w[0] * G.w[1]));
        double f[Q19], fs[Q19], F[3];
        for (int i = 0; i < Q19; ++i) f[i] = fin[(long)i * n + node];
        force_at(Fu, Ff, n, node, F);
        collide_node19(&k, f, F, fs);
        const int c[3] = {x, y, z};
        for (int i = 0; i < Q19; ++i) {
            const int ei[3] = {EX19[i], EY19[i], EZ19[i]};
            int l[3], partial = 0, beyond = 0;
            double uw[3] = {0.0, 0.0, 0.0};
            for (int a = 0; a < 3; ++a) {
                const int gc = G.o[a] + c[a] + ei[a];
                l[a] = locate(&G, a, gc);
                if (l[a] == -2) partial = 1;
                if (l[a] == -1) {
                    ++beyond;
                    if (wall_u)
                        for (int b = 0; b < 3; ++b) uw[b] += wall_u[3 * (2 * a + (gc < 0 ? 0 : 1)) + b];
                }
            }
            if (partial) continue;
            long tgt = -1;
            if (!beyond) {
                tgt = (long)l[0] + (long)G.w[0] * ((long)l[1] + (long)G.w[1] * l[2]);
                if (solid && solid[tgt]) tgt = -1;
            }
            if (tgt >= 0) {
                fout[(long)i * n + tgt] = fs[i];
            } else {
                double corr = 0.0;
                if (beyond)
                    corr = 2.0 * weight19(i) * (ei[0] * uw[0] + ei[1] * uw[1] + ei[2] * uw[2]) / (beyond * CS2);
                fout[(long)opp[i] * n + node] = fs[i] - corr;
            }
        }
    }
    return 0;
}

/* One D3Q19 time step with walls at rest. */
int orc19_step(const int *geom, const double *s, const double *Fu, const double *Ff,
               const uint8_t *solid, const double *fin, double *fout)
{
    return orc19_step_ex(geom, s, Fu, Ff, solid, NULL, fin, fout);
}

/* Eq. (9) on every D3Q19 node. */
int orc19_macro(const int *geom, const double *Fu, const double *Ff, const uint8_t *solid,
                const double *f, double *rho, double *u)
{
    orc_geom G;
    if (geom_read(geom, &G)) return 1;
    const long n = G.n;
#pragma omp parallel for schedule(static)
    for (long node = 0; node < n; ++node) {
        if (solid && solid[node]) {
            rho[node] = 0.0;
            u[node] = u[n + node] = u[2 * n + node] = 0.0;
            continue;
        }
        double fl[Q19], F[3], r, uu[3];
        for (int i = 0; i < Q19; ++i) fl[i] = f[(long)i * n + node];
        force_at(Fu, Ff, n, node, F);
        macro_node19(fl, F, &r, uu);
        rho[node] = r;
        u[node] = uu[0];
        u[n + node] = uu[1];
        u[2 * n + node] = uu[2];
    }
    return 0;
}

/* Initial D3Q19 state: f = f_eq(rho0(x), u0(x)). */
int orc19_init(const int *geom, const double *rho0, const double *u0, double *f)
{
    orc_geom G;
    if (geom_read(geom, &G)) return 1;
    const long n = G.n;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (long node = 0; node < n; ++node) {
        double u[3], fe[Q19];
        const double r = rho0 ? rho0[node] : 1.0;
        for (int a = 0; a < 3; ++a) u[a] = u0 ? u0[(long)a * n + node] : 0.0;
        bad |= orc19_equilibrium(r, u, fe);
        for (int i = 0; i < Q19; ++i) f[(long)i * n + node] = fe[i];
    }
    return bad ? 2 : 0;
}

/* ======================================================================== */
/* Non-orthogonal raw-moment MRT of Appendix B; moving walls                 */
/* ======================================================================== */
/*
 * MRT (Appendix B): the collision of Eq. (5) in raw-moment space, with the
 * raw moments T = M f of Eq. (14), the equilibria T_eq = M f_D^eq of the
 * discrete equilibrium f_D^eq = w rho [1 + e.u/c_s^2 + (e.u)^2/(2 c_s^4)
 * - u^2/(2 c_s^2)] (Sec. II B) and the forcing G = M R_G of Guo et al.,
 * R_G = w [(e - u)/c_s^2 + (e.u) e/c_s^4] . F:
 *     T* = T - S (T - T_eq) + (I - S/2) G,   f* = M^-1 T*,
 * with the same block-diagonal S (Eq. (13)) and u = (sum f e + F/2)/rho.
 *
 * Moving walls: a population leaving fluid node x along e_i through wall faces
 * moving with velocity u_w returns to x reversed with the momentum exchange of
 * a moving wall, f_opp(i)(x, t+1) = f*_i(x, t) - 2 w_i rho_w (e_i . u_w)/c_s^2,
 * rho_w = 1.  wall_u[6][3]: velocity of face (axis a, side s) at [2a + s],
 * side 0 the face below coordinate 0, side 1 the face beyond n_a - 1.  A link
 * that crosses several faces at once (edges, corners) takes the mean of their
 * velocities; links into solid nodes see a wall at rest.
 */
static double weight27(int i)
{
    const int k = abs(EX[i]) + abs(EY[i]) + abs(EZ[i]);
    return k == 0 ? 8.0 / 27.0 : (k == 1 ? 2.0 / 27.0 : (k == 2 ? 1.0 / 54.0 : 1.0 / 216.0));
}

/* discrete equilibrium f_D^eq (Sec. II B) */
void orc_mrt_feq(double rho, const double *u, double *feq)
{
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < Q; ++i) {
        const double eu = EX[i] * u[0] + EY[i] * u[1] + EZ[i] * u[2];
        feq[i] = weight27(i) * rho * (1.0 + eu / CS2 + eu * eu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
    }
}

/* Guo forcing term R_G (Appendix B) */
void orc_mrt_guo(const double *u, const double *F, double *R)
{
    for (int i = 0; i < Q; ++i) {
        const double e[3] = {(double)EX[i], (double)EY[i], (double)EZ[i]};
        const double eu = e[0] * u[0] + e[1] * u[1] + e[2] * u[2];
        double acc = 0.0;
        for (int a = 0; a < 3; ++a) acc += ((e[a] - u[a]) / CS2 + eu * e[a] / (CS2 * CS2)) * F[a];
        R[i] = weight27(i) * acc;
    }
}

typedef struct {
    double S[Q * Q];
    double M[Q * Q];
    double Minv[Q * Q];
} orc_mrt_consts;

static int mrt_consts_init(orc_mrt_consts *k, const double *s)
{
    orc_matrix_S(s, k->S);
    orc_matrix_M(k->M);
    return invert(Q, k->M, k->Minv);
}

static void mrt_collide_node(const orc_mrt_consts *k, const double *f, const double *F, double *fs)
{
    double rho, u[3], feq[Q], R[Q], T[Q], Teq[Q], G[Q], d[Q], Sd[Q], SG[Q], Ts[Q];
    macro_node(f, F, &rho, u);
    orc_mrt_feq(rho, u, feq);
    orc_mrt_guo(u, F, R);
    matvec(k->M, f, T);
    matvec(k->M, feq, Teq);
    matvec(k->M, R, G);
    for (int a = 0; a < Q; ++a) d[a] = T[a] - Teq[a];
    matvec(k->S, d, Sd);
    matvec(k->S, G, SG);
    for (int a = 0; a < Q; ++a) Ts[a] = T[a] - Sd[a] + G[a] - 0.5 * SG[a];
    matvec(k->Minv, Ts, fs);
}

int orc_mrt_collide(const double *f, const double *F, const double *s, double *fs)
{
    orc_mrt_consts k;
    if (mrt_consts_init(&k, s)) return 1;
    mrt_collide_node(&k, f, F, fs);
    return 0;
}

/*
 * One D3Q27 time step with a choice of collision (model 0: the cascaded scheme
 * of Sec. II, model 1: the MRT above) and moving walls (wall_u as above, or
 * NULL for walls at rest).  Other arguments as orc_step.
 */
int orc_step_ex(const int *geom, const double *s, const double *Fu, const double *Ff, const uint8_t *solid,
                const double *wall_u, int model, const double *fin, double *fout)
{
    orc_geom G;
    orc_consts kc;
    orc_mrt_consts km;
    if (geom_read(geom, &G)) return 1;
    if (model != 0 && model != 1) return 3;
    if (model == 0 ? consts_init(&kc, s) : mrt_consts_init(&km, s)) return 2;
    const long n = G.n;
    for (long idx = 0; idx < (long)Q * n; ++idx) fout[idx] = NAN;
    if (solid)
        for (long node = 0; node < n; ++node)
            if (solid[node])
                for (int i = 0; i < Q; ++i) fout[(long)i * n + node] = fin[(long)i * n + node];
    int opp[Q];
    for (int i = 0; i < Q; ++i) opp[i] = opposite(i);

#pragma omp parallel for schedule(static)
    for (long node = 0; node < n; ++node) {
        if (solid && solid[node]) continue;
        const int c[3] = {(int)(node % G.w[0]), (int)((node / G.w[0]) % G.w[1]),
                          (int)(node / ((long)G.w[0] * G.w[1]))};
        double f[Q], fs[Q], F[3];
        for (int i = 0; i < Q; ++i) f[i] = fin[(long)i * n + node];
        force_at(Fu, Ff, n, node, F);
        if (model == 0)
            collide_node(&kc, f, F, fs);
        else
            mrt_collide_node(&km, f, F, fs);
        for (int i = 0; i < Q; ++i) {
            const int ei[3] = {EX[i], EY[i], EZ[i]};
            int l[3], partial = 0, beyond = 0;
            double uw[3] = {0.0, 0.0, 0.0};
            for (int a = 0; a < 3; ++a) {
                const int gc = G.o[a] + c[a] + ei[a];
                l[a] = locate(&G, a, gc);
                if (l[a] == -2) partial = 1;
                if (l[a] == -1) {
                    const int side = gc < 0 ? 0 : 1;
                    ++beyond;
                    if (wall_u)
                        for (int b = 0; b < 3; ++b) uw[b] += wall_u[3 * (2 * a + side) + b];
                }
            }
            if (partial) continue;
            long tgt = -1;
            if (!beyond) {
                tgt = (long)l[0] + (long)G.w[0] * ((long)l[1] + (long)G.w[1] * l[2]);
                if (solid && solid[tgt]) tgt = -1;
            }
            if (tgt >= 0) {
                fout[(long)i * n + tgt] = fs[i];
            } else {
                double corr = 0.0;
                if (beyond)
                    corr = 2.0 * weight27(i) * (ei[0] * uw[0] + ei[1] * uw[1] + ei[2] * uw[2]) / (beyond * CS2);
                fout[(long)opp[i] * n + node] = fs[i] - corr;
            }
        }
    }
    return 0;
}

/* Initial state for the MRT: f = f_D^eq(rho0(x), u0(x)). */
int orc_mrt_init(const int *geom, const double *rho0, const double *u0, double *f)
{
    orc_geom G;
    if (geom_read(geom, &G)) return 1;
    const long n = G.n;
#pragma omp parallel for schedule(static)
    for (long node = 0; node < n; ++node) {
        double u[3], fe[Q];
        const double r = rho0 ? rho0[node] : 1.0;
        for (int a = 0; a < 3; ++a) u[a] = u0 ? u0[(long)a * n + node] : 0.0;
        orc_mrt_feq(r, u, fe);
        for (int i = 0; i < Q; ++i) f[(long)i * n + node] = fe[i];
    }
    return 0;
}

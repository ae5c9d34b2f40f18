/*
 * clbm.h -- C ABI of the MI355X (gfx950) D3Q27 cascaded lattice Boltzmann
 * library: the collide-and-stream update of Fei, Luo & Li, "Three-dimensional
 * cascaded lattice Boltzmann method: improved implementation and consistent
 * forcing scheme" (arXiv:1801.04586), its adjoint, and reduced-precision
 * population storage; also the D3Q19 variant of the paper's Appendix A.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Lattice: nx * ny * nz nodes, node id n = x + nx * (y + ny * z), x fastest.
 *    N = nx * ny * nz must be below 2^31, and N times the widest element a
 *    plane holds (8 bytes for CLBM_F64 storage, 4 otherwise: state, adjoint
 *    and force planes) must not exceed 4 GiB, since kernels address a plane
 *    with 32-bit byte offsets: N <= 2^29 for FP64, N <= 2^30 otherwise.
 *    Lattice units: dx = dt = 1, c_s^2 = 1/3 (Sec. II A).
 *  - Axes: wall[a] = 0 makes axis a periodic; wall[a] = 1 puts stationary
 *    half-way bounce-back walls at both ends of axis a (Sec. III): a population
 *    leaving fluid node x towards a wall or a solid node returns to x,
 *    reversed, one step later.  On a walled axis node j sits at coordinate
 *    j + 1/2 with walls at 0 and n.
 *  - Populations i = 0..Q-1 follow the velocity order of Eq. (1) (Q = 27) or
 *    of Eq. (A1) (Q = 19, lattice CLBM_D3Q19: the first 19 velocities of
 *    Eq. (1)).
 *  - Pointers are device pointers unless a comment says "host".  Every device
 *    buffer is allocated and freed by the caller; the library never frees
 *    caller memory.  Buffers must be 16-byte aligned.
 *  - All work is enqueued on the context's stream (a hipStream_t passed as
 *    void*, NULL = default stream) and is asynchronous, except where noted.
 *  - A context is not thread-safe; calls on one context must not overlap.
 *  - Every function returns a clbm_status; argument errors are detected on the
 *    host before any HIP call is made.  CLBM_EHIP carries the HIP error text in
 *    clbm_last_error().
 *
 * State buffers
 * -------------
 * A state is one array [Q][P] of the storage type, P = plane_stride of the
 * description (>= N; P = N when plane_stride is 0): plane i holds population i
 * of every node, node n at entry [i][n] ([Q][nz][ny][nx] when P = N); entries
 * n >= N are padding the library never reads or writes, except that
 * clbm_copy copies whole buffers.  A plane stride a few KiB above a power of
 * two keeps the Q planes of a large lattice from mapping onto the same HBM
 * channels (clbm_default_plane_stride).  Its contents are
 * the populations in "pull" order: entry [i][y] holds the pre-collision
 * population f_i(y + e_i, t) when y + e_i is a fluid node, and f_opp(i)(y, t)
 * (the one that bounces back into y) when the link from y along e_i is
 * blocked by a wall or a solid node.  Equivalently it holds the post-collision
 * populations f*_i(y, t-1) of Eq. (7) before the streaming of Eq. (8).
 * clbm_get_populations/clbm_set_populations convert from/to plain
 * pre-collision populations f(x, t).  Storage types:
 *    CLBM_F64  stores f_i itself, arithmetic in FP64;
 *    CLBM_F32, CLBM_F16, CLBM_BF16 store the deviation f_i - w_i from the
 *    rest-state weights (D3Q27: 8/27, 2/27, 1/54, 1/216; D3Q19: 1/3, 1/18,
 *    1/36), rounded to nearest even, arithmetic in FP32.
 * Entries belonging to solid nodes are never read; the step stores unspecified
 * values there (whole cache lines are written for speed).
 */
#ifndef CLBM_H
#define CLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CLBM_ABI_VERSION 7

/* Velocity sets: D3Q27 (Eq. (1), moment set Eq. (12)) and D3Q19 (Appendix A,
 * Eq. (A1)-(A6): velocities without the eight corners, moments of Eq. (A2),
 * rates s3 for the six third-order and s4 for the three fourth-order moments;
 * s3b, s4b, s5 and s6 are unused).  D3Q19 has no adjoint (clbm_adjoint_step and
 * clbm_loss_seed return CLBM_EINVAL); with FP32 or FP64 storage it takes fused
 * step pairs like D3Q27 (see clbm_run). */
typedef enum clbm_lattice {
    CLBM_D3Q27 = 0,
    CLBM_D3Q19 = 1
} clbm_lattice;

/* Collision models.  CLBM_CASCADED: the cascaded scheme of Sec. II (Eq. (5),
 * (13), (15), (16)).  CLBM_MRT: the non-orthogonal raw-moment MRT of
 * Appendix B on D3Q27 -- raw moments T = M f of Eq. (14), equilibria
 * M f_D^eq of the discrete equilibrium of Sec. II B, forcing M R_G of Guo et
 * al., T* = T - S (T - T_eq) + (I - S/2) G with the same S (Eq. (13)); its
 * initial state (clbm_init) is f_D^eq.  The MRT has no adjoint. */
typedef enum clbm_collision {
    CLBM_CASCADED = 0,
    CLBM_MRT = 1
} clbm_collision;

typedef enum clbm_dtype {
    CLBM_F64 = 0,
    CLBM_F32 = 1,
    CLBM_F16 = 2,
    CLBM_BF16 = 3
} clbm_dtype;

typedef enum clbm_status {
    CLBM_OK = 0,
    CLBM_EINVAL = 1,     /* bad dims, null/misaligned pointer, bad argument */
    CLBM_ERATE = 2,      /* a relaxation rate outside (0, 2) */
    CLBM_EDTYPE = 3,     /* unknown storage type */
    CLBM_EHIP = 4,       /* a HIP runtime call or kernel launch failed */
    CLBM_ENONFINITE = 5  /* clbm_moments found a non-finite value or rho <= 0 */
} clbm_status;

/* Static description of a lattice.  Rates and force can be changed later with
 * clbm_set_rates / clbm_set_force. */
typedef struct clbm_desc {
    int32_t nx, ny, nz;       /* >= 1 each, nx * ny * nz < 2^31 */
    int32_t wall[3];          /* per axis: 0 periodic, 1 half-way bounce-back walls */
    int32_t storage;          /* clbm_dtype */
    int32_t lattice;          /* clbm_lattice: CLBM_D3Q27 (0) or CLBM_D3Q19 (1) */
    /* Relaxation rates of Eq. (13), in this order:
     * s0, s1, s2 (= s_nu, shear: nu = (1/s2 - 1/2)/3), s2b (bulk:
     * xi = 2/3 (1/s2b - 1/2)/3), s3, s3b, s4, s4b, s5, s6.  Each in (0, 2). */
    double s[10];
    /* Body force density F(x) = force_uniform + force_scale * force[.][x]
     * (Eq. (6), (9), (16)).  force: device [3][N], FP64 for CLBM_F64 storage,
     * FP32 otherwise, or NULL. */
    double force_uniform[3];
    double force_scale;
    const void *force;
    /* Solid mask: device uint8 [N], nonzero = solid, or NULL (all fluid).  Read
     * once, by clbm_create, which derives the context's link table from it. */
    const uint8_t *solid;
    int32_t collision;        /* clbm_collision; CLBM_MRT needs CLBM_D3Q27 */
    int32_t reserved;         /* must be 0 */
    /* Velocities of the wall faces (host copy taken by clbm_create):
     * wall_velocity[2a + s] for axis a, side s = 0 the face below coordinate 0,
     * s = 1 the face beyond n_a - 1.  A population that leaves a fluid node
     * along e_i through moving faces returns reversed with the momentum
     * exchange -2 w_i (e_i . u_w)/c_s^2 (wall density 1), u_w the mean velocity
     * of the faces the link crosses; links into solid nodes see a wall at
     * rest.  Faces of periodic axes must have zero velocity.  All zero: the
     * walls of Sec. III, at rest (used for the lid-driven cavity of
     * Appendix B). */
    double wall_velocity[6][3];
    /* Plane stride P of state buffers in elements: 0 (P = N) or a value in
     * [N, 2^32) with P * element size a multiple of 16 bytes. */
    int64_t plane_stride;
} clbm_desc;

typedef struct clbm_ctx clbm_ctx;

/* Recommended plane stride for a lattice: N rounded up to 256 bytes plus 4 KiB
 * (Q-plane streams at power-of-two distances contend for the same HBM
 * channels; on MI355X the padded stride measured up to 8% faster at 512^3).
 * Returns -1 for invalid dims or storage.  Host only; no context needed. */
int64_t clbm_default_plane_stride(int32_t nx, int32_t ny, int32_t nz, int32_t storage);

/* ABI version of the loaded library (CLBM_ABI_VERSION). */
int clbm_abi_version(void);

/* Static text for a status code.  Never NULL. */
const char *clbm_strerror(int status);

/* Text of the last error on this context (may include HIP's message).  Never NULL. */
const char *clbm_last_error(const clbm_ctx *ctx);

/* Create a context for the lattice *desc (copied; the force buffer is
 * referenced, not copied, and must outlive its use).  stream: hipStream_t or
 * NULL.  Allocates device scratch for reductions (130 KiB; on D3Q27 cascaded
 * lattices, whose adjoint keeps one row of partial sums per 256 nodes, 0.26
 * bytes per node if that is more) and, when
 * desc->solid is given or the lattice has walls and FP32 or FP64 storage (the
 * storage types with fused step pairs, see clbm_run), a link table of 4 bytes
 * per node built from the solid mask
 * and the walls by a kernel enqueued on `stream` (the mask must be ready when
 * that kernel runs; it is not referenced afterwards).  *out is set to NULL on
 * error. */
int clbm_create(clbm_ctx **out, const clbm_desc *desc, void *stream);

/* Release the context and its scratch (synchronises its stream). NULL is a no-op. */
int clbm_destroy(clbm_ctx *ctx);

/* Change the stream subsequent calls enqueue on. */
int clbm_set_stream(clbm_ctx *ctx, void *stream);

/* Replace the ten relaxation rates of Eq. (13) (host array, order as in clbm_desc). */
int clbm_set_rates(clbm_ctx *ctx, const double *s);

/* Replace the body force: uniform (host, 3 doubles, or NULL = 0), per-node field
 * (device [3][N] as in clbm_desc, or NULL) and the scale applied to the field. */
int clbm_set_force(clbm_ctx *ctx, const double *uniform, const void *field, double scale);

/* Initial state: writes into `state` the populations f = f_eq(rho0, u0) of the
 * generalized local equilibrium (NM)^-1 T_eq (Sec. II B, Eq. (15)).
 * rho0: device FP64 [N] or NULL (rho = 1); u0: device FP64 [3][N] or NULL (u = 0). */
int clbm_init(clbm_ctx *ctx, void *state, const double *rho0, const double *u0);

/* One time step, Steps 1-4 of Sec. II B fused in one kernel: pull-stream with
 * bounce-back (Eq. (8)), rho and u (Eq. (9)), raw moments (Eq. (4), (14)),
 * central shift N(u), collision (Eq. (5), (13), (15), (16)), back-shift N^-1 and
 * M^-1 (Eq. (7)).  src and dst are distinct state buffers.  When every rate
 * above second order is exactly 1 (s3 = s3b = s4 = s4b = s5 = s6 = 1, as in the
 * simulations of Sec. III) the kernel forms only the moments up to second order:
 * Eq. (5) then sets the higher ones to equilibrium + C/2 whatever their value. */
int clbm_step(clbm_ctx *ctx, const void *src, void *dst);

/* nsteps steps from the state in a, using a and b as the two buffers; the
 * buffer that holds the final state is returned in *result (host, may be
 * NULL).  On lattices with FP32 or FP64 storage (D3Q27 with the cascaded
 * collision or the MRT of Appendix B, D3Q19; any walls, moving or not, and
 * solid nodes), pairs of steps run as one fused launch that keeps the
 * intermediate state on chip (bitwise the same result as two clbm_step calls)
 * when the lattice fills the device: its 32 x 12 (x, y) tile columns (32 x 16
 * for periodic FP64 lattices with the cascaded collision) times z chunks of 8
 * planes give at least two blocks per compute unit (CLBM_OPT_* flags override
 * this); otherwise every step is one clbm_step.  nsteps >= 0. */
int clbm_run(clbm_ctx *ctx, void *a, void *b, int32_t nsteps, void **result);

/* nsteps steps from the state in src, keeping every state (not in the paper; for the adjoint's
 * recomputation): states (host array of nsteps device state
 * buffers, distinct from src and from one another) gets the state after k + 1 steps in states[k]; src
 * is not modified.  Every step is one clbm_step launch (bitwise the same results), without
 * clbm_run's fused pairs, since every state has to be written anyway.  nsteps >= 0 (0: nothing
 * happens). */
int clbm_trajectory(clbm_ctx *ctx, const void *src, void *const *states, int32_t nsteps);

/* Option flags (clbm_set_options). */
#define CLBM_OPT_SINGLE_STEP 1u /* clbm_run launches one step at a time */
#define CLBM_OPT_FUSED_PAIRS 2u /* fused pairs on every lattice that allows them, whatever its size */

/* Set the CLBM_OPT_* flags of a context (default 0: fused pairs chosen by
 * lattice size).  Setting both flags is CLBM_EINVAL. */
int clbm_set_options(clbm_ctx *ctx, uint32_t options);

/* 1 when clbm_run on this context runs pairs of steps as fused launches, 0 when
 * it runs single steps, CLBM_EINVAL for a NULL ctx. */
int clbm_fused_pairs(const clbm_ctx *ctx);

/* Copy a whole state buffer, Q x P elements (checkpoints).  src and dst
 * distinct. */
int clbm_copy(clbm_ctx *ctx, const void *src, void *dst);

/* Macroscopic fields of Eq. (9) from a state: rho device FP64 [N] or NULL,
 * u device FP64 [3][N] or NULL (solid nodes get 0).  totals (host, 4 doubles)
 * or NULL: FP64 sums over fluid nodes of rho and rho*u (deterministic
 * two-pass reduction); n_bad (host) or NULL: number of fluid nodes with a
 * non-finite rho/u or rho <= 0.  When totals or n_bad is non-NULL the call
 * synchronises the stream and returns CLBM_ENONFINITE if n_bad > 0. */
int clbm_moments(clbm_ctx *ctx, const void *state, double *rho, double *u, double *totals, int64_t *n_bad);

/* Pre-collision populations f(x, t) of a state, as device FP64 [Q][N] in
 * Eq. (1) order (f itself, not the deviation).  Solid nodes get 0. */
int clbm_get_populations(clbm_ctx *ctx, const void *state, double *f);

/* Pre-collision populations of selected nodes: out (device FP64 [Q][count])
 * gets f_i at node nodes[k] (device int32 [count], node ids as above) in
 * column k.  Solid nodes give 0; ids outside [0, N) give NaN.  count >= 0. */
int clbm_sample_populations(clbm_ctx *ctx, const void *state, const int32_t *nodes, int32_t count, double *out);

/* Inverse of clbm_get_populations: writes into `state` the buffer whose
 * pre-collision populations are f (device FP64 [Q][N]); values are rounded to
 * the storage type.  Solid-node entries are left untouched. */
int clbm_set_populations(clbm_ctx *ctx, const double *f, void *state);

/* Adjoint of one time step (the exact transpose of clbm_step's map; not in the
 * paper).  state_t: the state buffer clbm_step read to go from t to t+1.
 * lam_next: dJ/df(t+1), lam_out: dJ/df(t), both [27][N] of the adjoint type
 * (FP64 for CLBM_F64 storage, FP32 otherwise), pre-collision populations in
 * Eq. (1) order, distinct buffers; zero on solid nodes.
 * dJdF: device [3][N] of the adjoint type or NULL; dJ/dF(x) of this step is
 * added to it.  dJds: device FP64 [10] or NULL; dJ/ds_k of this step (summed
 * over nodes in FP64, fixed order) is added to it.  D3Q27 cascaded scheme
 * only (moving walls allowed: their momentum exchange is a constant). */
int clbm_adjoint_step(clbm_ctx *ctx, const void *state_t, const void *lam_next, void *lam_out, void *dJdF,
                      double *dJds);

/* clbm_adjoint_step for callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  Same arguments, error behaviour and results
 * (bitwise) as clbm_adjoint_step, and the same kernels; the call makes no allocation of any kind.  Its
 * dJ/ds partial sums go to a static device array of 8.03 MiB instead of the context's scratch: the
 * library holds one such array on every device it runs on until the process ends, and clbm_create
 * looks up its address on the context's device.  That array limits the lattice to
 * clbm_adjoint_noalloc_max_nodes() = 2^25 nodes; larger lattices get CLBM_EINVAL.  All calls on one
 * device share the array, so calls that overlap on one device (several streams or threads) race and
 * must be serialised by the caller.  Nothing in it needs clearing between calls: a call reads only
 * entries it has written itself. */
int clbm_adjoint_step_noalloc(clbm_ctx *ctx, const void *state_t, const void *lam_next, void *lam_out,
                              void *dJdF, double *dJds);

/* Largest lattice (nx * ny * nz) clbm_adjoint_step_noalloc accepts: 2^25.  Host only. */
int64_t clbm_adjoint_noalloc_max_nodes(void);

/* Loss J = 1/2 sum over fluid nodes |u(x) - u_target(x)|^2 with u of Eq. (9)
 * evaluated on `state`.  u_target: device [3][N] of the adjoint type.
 * lam_out: dJ/df [27][N] (adjoint type), the seed of the adjoint recursion.
 * dJdF (device [3][N] or NULL): the direct dependence of u on F/2 is added.
 * J (device FP64 [1] or NULL): J is added to *J (FP64, fixed-order sum). */
int clbm_loss_seed(clbm_ctx *ctx, const void *state, const void *u_target, void *lam_out, void *dJdF, double *J);

#ifdef __cplusplus
}
#endif

#endif /* CLBM_H */

// Per-node arithmetic of the D3Q27 cascaded LBM (arXiv:1801.04586, Sec. II),
// written for registers: every loop is unrolled at compile time and every array
// index is a constant, so a node's 27 values never leave VGPRs.
//
// Tensor-slot convention.  A node's 27 values live in v[9*a + 3*b + c].
//  - As populations, (a, b, c) = (e_x + 1, e_y + 1, e_z + 1).
//  - As moments, (a, b, c) = (m, n, p), the exponents of k_mnp (Eq. (2)).
// The moment set of Eq. (12) is exactly {0,1,2}^3, so M (Eq. (14)) and the shift
// N(u) (Eq. (4)) are tensor products of one 3x3 matrix per axis:
//   M1 = [[1,1,1],[-1,0,1],[1,0,1]] on (f(e=-1), f(0), f(+1)),
//   N1(u) = [[1,0,0],[-u,1,0],[u^2,-2u,1]],  N1(u)^-1 = N1(-u),
// and M, M^-1, N, N^-1 are applied as three passes of nine 3-vectors each.
// This is the split of the reconstruction into N^-1 then M^-1 that Sec. II B
// recommends, carried one level further (per axis).
//
// Deviation form.  Populations are handled as deviations d = f - w from the
// rest-state weights w = w1 (x) w1 (x) w1, w1 = (1/6, 2/3, 1/6).  The raw moments
// of w are E = e (x) e (x) e with e = (1, 0, 1/3), which are also the per-unit-
// density equilibria of Eq. (15).  With rho = 1 + drho and the central moments of
// w about u equal to c(ux) (x) c(uy) (x) c(uz), c(u) = (1, -u, 1/3 + u^2), every
// quantity the collision needs is formed from small numbers (drho, u, F, d), so
// FP32 arithmetic on FP32/FP16/BF16 deviations keeps its relative precision.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace clbm {

// ------------------------------------------------------------------ compile-time loops
template <int B, int E, typename F>
__device__ __forceinline__ void sfor(F &&f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        sfor<B + 1, E>(f);
    }
}

__host__ __device__ constexpr int slot(int a, int b, int c) { return 9 * a + 3 * b + c; }
__host__ __device__ constexpr int sa(int t) { return t / 9; }
__host__ __device__ constexpr int sb(int t) { return (t / 3) % 3; }
__host__ __device__ constexpr int sc(int t) { return t % 3; }

// Population index in the order of Eq. (1) for the velocity held in tensor slot t.
__host__ __device__ constexpr int pop_of_slot(int t)
{
    constexpr int tab[27] = {26, 10, 22, 14, 2, 12, 24, 8, 20, 18, 4, 16, 6, 0,
                             5,  17, 3,  15, 25, 9, 21, 13, 1, 11, 23, 7, 19};
    return tab[t];
}

// Velocity set of Eq. (1), typed here to cross-check the table above at compile time.
namespace eq1 {
constexpr int ex[27] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1};
constexpr int ey[27] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, 1, -1, -1, 1, 1, -1, -1};
constexpr int ez[27] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1, 1, 1, 1, 1, -1, -1, -1, -1};
constexpr bool table_ok()
{
    for (int t = 0; t < 27; ++t) {
        const int i = pop_of_slot(t);
        if (ex[i] != sa(t) - 1 || ey[i] != sb(t) - 1 || ez[i] != sc(t) - 1) return false;
    }
    return true;
}
static_assert(table_ok(), "slot -> population table disagrees with Eq. (1)");
}  // namespace eq1

// Rest-state weight of the velocity in slot t: product of (1/6, 2/3, 1/6) per axis.
template <typename R>
__host__ __device__ constexpr R weight_of_slot(int t)
{
    constexpr double w1[3] = {1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0};
    return R(w1[sa(t)] * w1[sb(t)] * w1[sc(t)]);
}

// ------------------------------------------------------------------ D3Q19 (Appendix A)
// The 19 velocities of Eq. (A1) are the first 19 of Eq. (1): every tensor slot
// except the eight corners, whose three components are all nonzero.  The moment
// set of Eq. (A2) is {0,1,2}^3 minus the eight triples whose exponents are all
// >= 1; it contains every triple below each of its members, so the shift N(u)
// and its inverse restricted to it need no other moment.
__host__ __device__ constexpr bool corner_population(int t) { return sa(t) != 1 && sb(t) != 1 && sc(t) != 1; }
__host__ __device__ constexpr bool outside_q19_moments(int t) { return sa(t) >= 1 && sb(t) >= 1 && sc(t) >= 1; }

namespace eqa1 {
constexpr bool table_ok()
{
    for (int t = 0; t < 27; ++t)
        if ((pop_of_slot(t) < 19) == corner_population(t)) return false;
    return true;
}
static_assert(table_ok(), "the D3Q19 velocities must be the first 19 populations of Eq. (1)");
}  // namespace eqa1

// Rest-state weight of the velocity in slot t on lattice Q (27 or 19).  D3Q19:
// 1/3 (rest), 1/18 (faces), 1/36 (edges), 0 for the absent corners.
template <int Q, typename R>
__host__ __device__ constexpr R lattice_weight(int t)
{
    if constexpr (Q == 27) {
        return weight_of_slot<R>(t);
    } else {
        const int k = (sa(t) != 1) + (sb(t) != 1) + (sc(t) != 1);
        return R(k == 0 ? 1.0 / 3.0 : (k == 1 ? 1.0 / 18.0 : (k == 2 ? 1.0 / 36.0 : 0.0)));
    }
}

// Does lattice Q have a population in slot t?
template <int Q>
__host__ __device__ constexpr bool has_slot(int t)
{
    return Q == 27 || !corner_population(t);
}

// e = (1, 0, 1/3): raw moments of w1, i.e. the equilibria of Eq. (15) per unit density.
__host__ __device__ constexpr double e_of(int k) { return k == 0 ? 1.0 : (k == 1 ? 0.0 : 1.0 / 3.0); }

// ------------------------------------------------------------------ relaxation rates
// Eq. (13).  s[] = {s0, s1, s2 (= s_nu), s2b, s3, s3b, s4, s4b, s5, s6}; hs = 1 - s/2;
// sm = s_- = (s2b - s2)/3 couples the three normal second moments.
template <typename R>
struct Rates {
    R s[10];
    R hs[10];
    R sm;
};

enum { R_S0 = 0, R_S1, R_S2, R_S2B, R_S3, R_S3B, R_S4, R_S4B, R_S5, R_S6 };

// Rate index of moment (m, n, p) of Eq. (12) outside the conserved slots and the
// normal-stress block.
__host__ __device__ constexpr int rate_of(int m, int n, int p)
{
    const int ones = (m == 1) + (n == 1) + (p == 1);
    const int order = m + n + p;
    if (order == 2) return R_S2;               // k110, k101, k011 (s_nu)
    if (order == 3 && ones == 1) return R_S3;  // k120 ... k021
    if (order == 3) return R_S3B;              // k111
    if (order == 4 && ones == 0) return R_S4;  // k220, k202, k022
    if (order == 4) return R_S4B;              // k211, k121, k112
    if (order == 5) return R_S5;               // k122, k212, k221
    return R_S6;                               // k222
}

// ------------------------------------------------------------------ per-axis passes
// Apply op(v0, v1, v2) to the nine triples along axis AX (0 = x, 1 = y, 2 = z).
template <int AX, typename R, typename Op>
__device__ __forceinline__ void axis_pass(R (&v)[27], Op &&op)
{
    sfor<0, 9>([&](auto K) {
        constexpr int k = decltype(K)::value;
        constexpr int o1 = k / 3, o2 = k % 3;
        constexpr int base = AX == 0 ? slot(0, o1, o2) : (AX == 1 ? slot(o1, 0, o2) : slot(o1, o2, 0));
        constexpr int st = AX == 0 ? 9 : (AX == 1 ? 3 : 1);
        op(v[base], v[base + st], v[base + 2 * st]);
    });
}

// M1: (f(-1), f(0), f(+1)) -> (k0, k1, k2) raw moments along one axis.
template <typename R>
__device__ __forceinline__ void raw_moments(R (&v)[27])
{
    auto op = [](R &a, R &b, R &c) {
        const R k0 = a + b + c, k1 = c - a, k2 = c + a;
        a = k0;
        b = k1;
        c = k2;
    };
    axis_pass<2>(v, op);
    axis_pass<1>(v, op);
    axis_pass<0>(v, op);
}

// N1(u): raw (k0, k1, k2) -> central (k0, k1 - u k0, k2 - 2u k1 + u^2 k0).
template <typename R>
__device__ __forceinline__ void shift_pass_op(R &k0, R &k1, R &k2, R u)
{
    const R t1 = fma(-u, k0, k1);
    k2 = fma(-u, k1 + t1, k2);
    k1 = t1;
}

template <typename R>
__device__ __forceinline__ void central_shift(R (&v)[27], R ux, R uy, R uz)
{
    axis_pass<0>(v, [=](R &a, R &b, R &c) { shift_pass_op(a, b, c, ux); });
    axis_pass<1>(v, [=](R &a, R &b, R &c) { shift_pass_op(a, b, c, uy); });
    axis_pass<2>(v, [=](R &a, R &b, R &c) { shift_pass_op(a, b, c, uz); });
}

// N1(-u): central (k0, k1, k2) -> raw (k0, k1 + u k0, k2 + 2u k1 + u^2 k0).
template <typename R>
__device__ __forceinline__ void unshift_pass_op(R &k0, R &k1, R &k2, R u)
{
    const R r1 = fma(u, k0, k1);
    k2 = fma(u, k1 + r1, k2);
    k1 = r1;
}

template <typename R>
__device__ __forceinline__ void central_unshift(R (&v)[27], R ux, R uy, R uz)
{
    axis_pass<0>(v, [=](R &a, R &b, R &c) { unshift_pass_op(a, b, c, ux); });
    axis_pass<1>(v, [=](R &a, R &b, R &c) { unshift_pass_op(a, b, c, uy); });
    axis_pass<2>(v, [=](R &a, R &b, R &c) { unshift_pass_op(a, b, c, uz); });
}

// N1(-u) followed by M1^-1: central (k0, k1, k2) -> populations
// (f(-1), f(0), f(+1)) = ((r2 - r1)/2, k0 - r2, (r2 + r1)/2).
template <typename R>
__device__ __forceinline__ void reconstruct(R (&v)[27], R ux, R uy, R uz)
{
    auto mk = [](R u) {
        return [=](R &k0, R &k1, R &k2) {
            const R r1 = fma(u, k0, k1);
            const R r2 = fma(u, k1 + r1, k2);
            const R h2 = R(0.5) * r2;
            const R fm = fma(R(-0.5), r1, h2);
            const R fp = fma(R(0.5), r1, h2);
            const R f0 = k0 - r2;
            k0 = fm;
            k1 = f0;
            k2 = fp;
        };
    };
    axis_pass<0>(v, mk(ux));
    axis_pass<1>(v, mk(uy));
    axis_pass<2>(v, mk(uz));
}

// D3Q19: post-collision central moments -> populations (Appendix A, Eq. (7)).
// N^-1 first (its rows for the moments of Eq. (A2) use only those moments); the
// raw moments outside the set, which vanish for any distribution on the 19
// velocities, are then set to zero, so that M^-1 of the full tensor set (three
// passes of M1^-1) returns exactly zero in the eight corner slots.
// M^-1 as three passes of M1^-1: raw (k0, k1, k2) -> (f(-1), f(0), f(+1)) =
// ((k2 - k1)/2, k0 - k2, (k2 + k1)/2) along each axis.
template <typename R>
__device__ __forceinline__ void inverse_raw_moments(R (&v)[27])
{
    auto op = [](R &k0, R &k1, R &k2) {
        const R h2 = R(0.5) * k2;
        const R fm = fma(R(-0.5), k1, h2);
        const R fp = fma(R(0.5), k1, h2);
        const R f0 = k0 - k2;
        k0 = fm;
        k1 = f0;
        k2 = fp;
    };
    axis_pass<0>(v, op);
    axis_pass<1>(v, op);
    axis_pass<2>(v, op);
}

template <typename R>
__device__ __forceinline__ void reconstruct_q19(R (&v)[27], R ux, R uy, R uz)
{
    central_unshift(v, ux, uy, uz);
    sfor<0, 27>([&](auto T) {
        if constexpr (outside_q19_moments(decltype(T)::value)) v[decltype(T)::value] = R(0);
    });
    inverse_raw_moments(v);
}

// ------------------------------------------------------------------ per-node velocity factors
// For one axis: q = c - e and c, the central moments of w1 about u, per exponent k.
template <typename R>
struct AxisU {
    R u, u2, c2;  // u, u^2, 1/3 + u^2
    __device__ __forceinline__ explicit AxisU(R u_) : u(u_), u2(u_ * u_), c2(R(1.0 / 3.0) + u_ * u_) {}
    template <int K>
    __device__ __forceinline__ R q() const { return K == 0 ? R(0) : (K == 1 ? -u : u2); }
    template <int K>
    __device__ __forceinline__ R c() const { return K == 0 ? R(1) : (K == 1 ? -u : c2); }
};

// G(m,n,p) = c_m c_n c_p - e_m e_n e_p, expanded so that no O(1) terms cancel:
// q_m c_n c_p + e_m q_n c_p + e_m e_n q_p.
template <int M, int N, int P, typename R>
__device__ __forceinline__ R g_term(const AxisU<R> &X, const AxisU<R> &Y, const AxisU<R> &Z)
{
    R g = R(0);
    if constexpr (M != 0) g = X.template q<M>() * Y.template c<N>() * Z.template c<P>();
    if constexpr (M != 1 && N != 0) g += R(e_of(M)) * Y.template q<N>() * Z.template c<P>();
    if constexpr (M != 1 && N != 1 && P != 0) g += R(e_of(M) * e_of(N)) * Z.template q<P>();
    return g;
}

// Full central moment of w about u: c_m c_n c_p.
template <int M, int N, int P, typename R>
__device__ __forceinline__ R cw_term(const AxisU<R> &X, const AxisU<R> &Y, const AxisU<R> &Z)
{
    return X.template c<M>() * Y.template c<N>() * Z.template c<P>();
}

// ------------------------------------------------------------------ collision (Eq. (5))
// On entry v holds the central moments of d about u; on exit the post-collision
// central moments minus those of w, T~* - N(u) M w, ready for reconstruct().
//   T~*   = T~ - S (T~ - rho E) + (I - S/2) C          (Eq. (5), (15), (16))
//   slot 000: T~* = rho; first-order slots: T~* = F/2 (the conserved moments;
//   their rates s0, s1 drop out exactly).
template <typename R>
__device__ __forceinline__ void collide(R (&v)[27], R drho, const AxisU<R> &X, const AxisU<R> &Y,
                                        const AxisU<R> &Z, R Fx, R Fy, R Fz, const Rates<R> &s)
{
    constexpr R cs2 = R(1.0 / 3.0), cs4 = R(1.0 / 9.0);
    sfor<0, 27>([&](auto T) {
        constexpr int t = decltype(T)::value;
        constexpr int m = sa(t), n = sb(t), p = sc(t);
        constexpr int ones = (m == 1) + (n == 1) + (p == 1);
        constexpr int order = m + n + p;
        if constexpr (order == 0) {
            v[t] = drho;
        } else if constexpr (order == 1) {
            // T~*_100 = F_x/2, minus the w part c_1(u_x) = -u_x
            v[t] = m == 1 ? fma(R(0.5), Fx, X.u) : (n == 1 ? fma(R(0.5), Fy, Y.u) : fma(R(0.5), Fz, Z.u));
        } else if constexpr (order == 2 && ones == 0) {
            // normal second moments: relaxed below as a block
        } else {
            constexpr int k = rate_of(m, n, p);
            constexpr R E = R(e_of(m) * e_of(n) * e_of(p));
            R neq = v[t] + g_term<m, n, p>(X, Y, Z);
            if constexpr (ones == 0) neq = fma(-drho, E, neq);
            R out = fma(-s.s[k], neq, v[t]);
            if constexpr (ones == 1) {
                // Eq. (16): F_alpha c_s^(m+n+p-1) in the slot whose single odd exponent is alpha
                constexpr R cf = order == 3 ? cs2 : cs4;
                const R Fa = m == 1 ? Fx : (n == 1 ? Fy : Fz);
                out = fma(s.hs[k] * cf, Fa, out);
            }
            v[t] = out;
        }
    });
    // block of Eq. (13) on (k200, k020, k002): deviators at s2, trace at s2b
    constexpr int ix = slot(2, 0, 0), iy = slot(0, 2, 0), iz = slot(0, 0, 2);
    const R nx = v[ix] + X.u2 - drho * cs2;
    const R ny = v[iy] + Y.u2 - drho * cs2;
    const R nz = v[iz] + Z.u2 - drho * cs2;
    const R tr = s.sm * (nx + ny + nz);
    v[ix] -= fma(s.s[R_S2], nx, tr);
    v[iy] -= fma(s.s[R_S2], ny, tr);
    v[iz] -= fma(s.s[R_S2], nz, tr);
}

// Collision when every rate above second order is one (s3 = s3b = s4 = s4b = s5 =
// s6 = 1, the setting of the paper's simulations, Sec. III).  Eq. (5) then sets
// each central moment of order >= 3 to its equilibrium plus C/2, independently
// of the pre-collision value, so only the raw and central moments up to second
// order are formed.  On entry v holds the deviations d (populations); on exit
// the post-collision central moments minus those of w, as collide() leaves them.
template <typename R>
__device__ __forceinline__ void collide_high1(R (&v)[27], R Fx, R Fy, R Fz, const Rates<R> &s, R &ux_out, R &uy_out,
                                              R &uz_out)
{
    constexpr R cs2 = R(1.0 / 3.0), cs4 = R(1.0 / 9.0);
    // z pass, complete: v[slot(a, b, p)] = moment p along z of the (a, b) column
    axis_pass<2>(v, [](R &a, R &b, R &c) {
        const R k0 = a + b + c, k1 = c - a, k2 = c + a;
        a = k0;
        b = k1;
        c = k2;
    });
    // y pass: only (n, p) with n + p <= 2 are needed
    R Y[3][3][3];  // [a][n][p]
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const R m0 = v[slot(a, 0, 0)], z0 = v[slot(a, 1, 0)], p0 = v[slot(a, 2, 0)];
        Y[a][0][0] = m0 + z0 + p0;
        Y[a][1][0] = p0 - m0;
        Y[a][2][0] = p0 + m0;
        const R m1 = v[slot(a, 0, 1)], z1 = v[slot(a, 1, 1)], p1 = v[slot(a, 2, 1)];
        Y[a][0][1] = m1 + z1 + p1;
        Y[a][1][1] = p1 - m1;
        Y[a][0][2] = v[slot(a, 0, 2)] + v[slot(a, 1, 2)] + v[slot(a, 2, 2)];
    }
    // x pass: raw moments T_d(m, n, p) with m + n + p <= 2
    const R t000 = Y[0][0][0] + Y[1][0][0] + Y[2][0][0];
    const R t100 = Y[2][0][0] - Y[0][0][0];
    const R t200 = Y[2][0][0] + Y[0][0][0];
    const R t010 = Y[0][1][0] + Y[1][1][0] + Y[2][1][0];
    const R t110 = Y[2][1][0] - Y[0][1][0];
    const R t001 = Y[0][0][1] + Y[1][0][1] + Y[2][0][1];
    const R t101 = Y[2][0][1] - Y[0][0][1];
    const R t011 = Y[0][1][1] + Y[1][1][1] + Y[2][1][1];
    const R t020 = Y[0][2][0] + Y[1][2][0] + Y[2][2][0];
    const R t002 = Y[0][0][2] + Y[1][0][2] + Y[2][0][2];
    // Eq. (9)
    const R drho = t000;
    // correctly rounded: with the hardware reciprocal (1 ulp) the FP32-storage velocity error of the
    // 128^3 Taylor-Green run after 1000 steps grew from below 1e-5 to 1.5e-5 relative
    const R inv_rho = R(1) / (R(1) + drho);
    const R ux = (t100 + R(0.5) * Fx) * inv_rho;
    const R uy = (t010 + R(0.5) * Fy) * inv_rho;
    const R uz = (t001 + R(0.5) * Fz) * inv_rho;
    ux_out = ux;
    uy_out = uy;
    uz_out = uz;
    const AxisU<R> X(ux), Y_(uy), Z(uz);
    // central second moments of d about u (N(u) restricted to order 2)
    const R c200 = fma(ux, fma(ux, t000, R(-2) * t100), t200);
    const R c020 = fma(uy, fma(uy, t000, R(-2) * t010), t020);
    const R c002 = fma(uz, fma(uz, t000, R(-2) * t001), t002);
    const R c110 = fma(ux * uy, t000, fma(-ux, t010, fma(-uy, t100, t110)));
    const R c101 = fma(ux * uz, t000, fma(-ux, t001, fma(-uz, t100, t101)));
    const R c011 = fma(uy * uz, t000, fma(-uy, t001, fma(-uz, t010, t011)));
    // post-collision central moments minus those of w
    sfor<0, 27>([&](auto T) {
        constexpr int t = decltype(T)::value;
        constexpr int m = sa(t), n = sb(t), p = sc(t);
        constexpr int ones = (m == 1) + (n == 1) + (p == 1);
        constexpr int order = m + n + p;
        if constexpr (order == 0) {
            v[t] = drho;
        } else if constexpr (order == 1) {
            v[t] = m == 1 ? fma(R(0.5), Fx, ux) : (n == 1 ? fma(R(0.5), Fy, uy) : fma(R(0.5), Fz, uz));
        } else if constexpr (order == 2 && ones == 2) {
            const R c = m == 0 ? c011 : (n == 0 ? c101 : c110);
            const R neq = c + g_term<m, n, p>(X, Y_, Z);
            v[t] = fma(-s.s[R_S2], neq, c);
        } else if constexpr (order >= 3) {
            // equilibrium + C/2: drho E - G + C/2
            constexpr R E = R(e_of(m) * e_of(n) * e_of(p));
            R out = -g_term<m, n, p>(X, Y_, Z);
            if constexpr (ones == 0) out = fma(drho, E, out);
            if constexpr (ones == 1) {
                constexpr R cf = R(0.5) * (order == 3 ? cs2 : cs4);
                out = fma(cf, m == 1 ? Fx : (n == 1 ? Fy : Fz), out);
            }
            v[t] = out;
        }
    });
    // block of Eq. (13) on (k200, k020, k002)
    const R nx = c200 + X.u2 - drho * cs2;
    const R ny = c020 + Y_.u2 - drho * cs2;
    const R nz = c002 + Z.u2 - drho * cs2;
    const R tr = s.sm * (nx + ny + nz);
    v[slot(2, 0, 0)] = c200 - fma(s.s[R_S2], nx, tr);
    v[slot(0, 2, 0)] = c020 - fma(s.s[R_S2], ny, tr);
    v[slot(0, 0, 2)] = c002 - fma(s.s[R_S2], nz, tr);
}

// ------------------------------------------------------------------ raw-moment MRT (Appendix B)
// Sum over the D3Q27 weights of e^k along one axis: 1, 0, 1/3, 0, 1/3 for k = 0..4.
__host__ __device__ constexpr double axis_moment(int k) { return k == 0 ? 1.0 : (k % 2 ? 0.0 : 1.0 / 3.0); }
__host__ __device__ constexpr double weight_moment(int m, int n, int p)
{
    return axis_moment(m) * axis_moment(n) * axis_moment(p);
}
__host__ __device__ constexpr int bump(int k, int axis, int a) { return k + (axis == a ? 1 : 0); }

// Raw moment (m, n, p) of sum_i w_i e_i^(mnp) (e_i . u)^ and (e_i . u)(e_i . V):
// first[a] = W(e + 1_a), second[a][b] = W(e + 1_a + 1_b), with W the weight moment.
template <int M, int N, int P, typename R>
__device__ __forceinline__ R weighted_dot1(const R (&u)[3])
{
    R acc = R(0);
    sfor<0, 3>([&](auto A) {
        constexpr int a = decltype(A)::value;
        constexpr double c = weight_moment(bump(M, 0, a), bump(N, 1, a), bump(P, 2, a));
        if constexpr (c != 0.0) acc = fma(R(c), u[a], acc);
    });
    return acc;
}
template <int M, int N, int P, typename R>
__device__ __forceinline__ R weighted_dot2(const R (&u)[3], const R (&V)[3])
{
    R acc = R(0);
    sfor<0, 3>([&](auto A) {
        constexpr int a = decltype(A)::value;
        sfor<0, 3>([&](auto B) {
            constexpr int b = decltype(B)::value;
            constexpr double c =
                weight_moment(bump(bump(M, 0, a), 0, b), bump(bump(N, 1, a), 1, b), bump(bump(P, 2, a), 2, b));
            if constexpr (c != 0.0) acc = fma(R(c) * u[a], V[b], acc);
        });
    });
    return acc;
}

// The non-orthogonal MRT of Appendix B on one node's deviations d = f - w, in
// place: raw moments T = M f (Eq. (14)), equilibria T_eq = M f_D^eq of the
// discrete equilibrium (Sec. II B), Guo forcing G = M R_G,
//     T* = T - S (T - T_eq) + (I - S/2) G,  f* = M^-1 T*,
// with the block S of Eq. (13) and u = (sum f e + F/2)/rho.  The raw moments of
// f_D^eq and R_G are closed forms in the weight moments of D3Q27:
//   M f_D^eq = rho [ (1 - u^2/(2 c_s^2)) W(e) + W1(u)/c_s^2 + W2(u, u)/(2 c_s^4) ],
//   M R_G    = (W1(F) - (u.F) W(e))/c_s^2 + W2(u, F)/c_s^4.
template <typename R>
__device__ __forceinline__ void collide_mrt(R (&v)[27], R Fx, R Fy, R Fz, const Rates<R> &s)
{
    raw_moments(v);  // deviation raw moments T - W
    const R drho = v[slot(0, 0, 0)];
    const R rho = R(1) + drho;
    const R inv_rho = R(1) / rho;
    const R u[3] = {(v[slot(1, 0, 0)] + R(0.5) * Fx) * inv_rho, (v[slot(0, 1, 0)] + R(0.5) * Fy) * inv_rho,
                    (v[slot(0, 0, 1)] + R(0.5) * Fz) * inv_rho};
    const R F[3] = {Fx, Fy, Fz};
    const R uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const R uF = u[0] * Fx + u[1] * Fy + u[2] * Fz;
    R neq[3], gb[3];
    sfor<0, 27>([&](auto T) {
        constexpr int t = decltype(T)::value;
        constexpr int m = sa(t), n = sb(t), p = sc(t);
        constexpr int ones = (m == 1) + (n == 1) + (p == 1);
        constexpr int order = m + n + p;
        if constexpr (order == 0) {
            // mass is conserved
        } else if constexpr (order == 1) {
            v[t] += m == 1 ? Fx : (n == 1 ? Fy : Fz);  // T* = T + F for any s1
        } else {
            constexpr R W = R(weight_moment(m, n, p));
            // equilibrium minus W: rho (3 W1 + 4.5 W2 - 1.5 u^2 W) + drho W
            R teq = fma(R(3), weighted_dot1<m, n, p>(u), R(4.5) * weighted_dot2<m, n, p>(u, u));
            if constexpr (W != R(0)) teq = fma(R(-1.5) * uu, W, teq);
            teq *= rho;
            if constexpr (W != R(0)) teq = fma(drho, W, teq);
            R g = fma(R(3), weighted_dot1<m, n, p>(F), R(9) * weighted_dot2<m, n, p>(u, F));
            if constexpr (W != R(0)) g = fma(R(-3) * uF, W, g);
            if constexpr (order == 2 && ones == 0) {
                constexpr int b = m == 2 ? 0 : (n == 2 ? 1 : 2);
                neq[b] = v[t] - teq;
                gb[b] = g;
            } else {
                constexpr int k = rate_of(m, n, p);
                const R out = fma(-s.s[k], v[t] - teq, v[t]);
                v[t] = fma(s.hs[k], g, out);
            }
        }
    });
    // block of Eq. (13) on (k200, k020, k002), for both the relaxation and (I - S/2) G
    const R nsum = s.sm * (neq[0] + neq[1] + neq[2]);
    const R gsum = s.sm * (gb[0] + gb[1] + gb[2]);
    constexpr int ib[3] = {slot(2, 0, 0), slot(0, 2, 0), slot(0, 0, 2)};
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const R sg = fma(s.s[R_S2], gb[b], gsum);
        v[ib[b]] = v[ib[b]] - fma(s.s[R_S2], neq[b], nsum) + gb[b] - R(0.5) * sg;
    }
    inverse_raw_moments(v);
}

// Deviation of the discrete equilibrium f_D^eq (Sec. II B) from w, per slot:
// w [drho (1 + ...) + 3 e.u + 4.5 (e.u)^2 - 1.5 u^2].
template <typename R>
__device__ __forceinline__ void discrete_equilibrium_dev(R (&v)[27], R drho, R ux, R uy, R uz)
{
    const R uu = ux * ux + uy * uy + uz * uz;
    sfor<0, 27>([&](auto T) {
        constexpr int t = decltype(T)::value;
        const R eu = R(sa(t) - 1) * ux + R(sb(t) - 1) * uy + R(sc(t) - 1) * uz;
        const R poly = fma(R(3), eu, fma(R(4.5) * eu, eu, R(-1.5) * uu));
        v[t] = weight_of_slot<R>(t) * fma(drho, R(1) + poly, poly);
    });
}

// Deviation of the generalized equilibrium (Sec. II B) in central-moment space:
// T_eq - N(u) M w = drho E - G.  Feeding it to reconstruct() gives f_eq - w.
template <typename R>
__device__ __forceinline__ void equilibrium_moments(R (&v)[27], R drho, const AxisU<R> &X, const AxisU<R> &Y,
                                                    const AxisU<R> &Z)
{
    sfor<0, 27>([&](auto T) {
        constexpr int t = decltype(T)::value;
        constexpr int m = sa(t), n = sb(t), p = sc(t);
        constexpr R E = R(e_of(m) * e_of(n) * e_of(p));
        v[t] = drho * E - g_term<m, n, p>(X, Y, Z);
    });
}

// ------------------------------------------------------------------ transposed passes (adjoint)
// (M1^-1)^T: adjoint of populations (a-, a0, a+) -> adjoint of raw (r0, r1, r2).
template <typename R>
__device__ __forceinline__ void reconstruct_raw_T(R (&v)[27])
{
    auto op = [](R &am, R &a0, R &ap) {
        const R r0 = a0;
        const R r1 = R(0.5) * (ap - am);
        const R r2 = fma(R(0.5), am + ap, -a0);
        am = r0;
        a0 = r1;
        ap = r2;
    };
    axis_pass<0>(v, op);
    axis_pass<1>(v, op);
    axis_pass<2>(v, op);
}

// N1(-u)^T: adjoint of raw (r0, r1, r2) -> adjoint of central (k0, k1, k2).
template <typename R>
__device__ __forceinline__ void unshift_T(R (&v)[27], R ux, R uy, R uz)
{
    auto mk = [](R u) {
        return [=](R &r0, R &r1, R &r2) {
            const R k0 = fma(u, fma(u, r2, r1), r0);  // r0 + u r1 + u^2 r2
            const R k1 = fma(R(2) * u, r2, r1);        // r1 + 2u r2
            r0 = k0;
            r1 = k1;
        };
    };
    axis_pass<0>(v, mk(ux));
    axis_pass<1>(v, mk(uy));
    axis_pass<2>(v, mk(uz));
}

// N1(u)^T: adjoint of central (k0, k1, k2) -> adjoint of raw (r0, r1, r2).
template <typename R>
__device__ __forceinline__ void shift_T(R (&v)[27], R ux, R uy, R uz)
{
    auto mk = [](R u) {
        return [=](R &k0, R &k1, R &k2) {
            const R r0 = fma(-u, fma(-u, k2, k1), k0);  // k0 - u k1 + u^2 k2
            const R r1 = fma(R(-2) * u, k2, k1);         // k1 - 2u k2
            k0 = r0;
            k1 = r1;
        };
    };
    axis_pass<0>(v, mk(ux));
    axis_pass<1>(v, mk(uy));
    axis_pass<2>(v, mk(uz));
}

// M1^T: adjoint of raw (k0, k1, k2) -> adjoint of populations (f(-1), f(0), f(+1)).
template <typename R>
__device__ __forceinline__ void raw_moments_T(R (&v)[27])
{
    auto op = [](R &k0, R &k1, R &k2) {
        const R fm = k0 - k1 + k2, f0 = k0, fp = k0 + k1 + k2;
        k0 = fm;
        k1 = f0;
        k2 = fp;
    };
    axis_pass<0>(v, op);
    axis_pass<1>(v, op);
    axis_pass<2>(v, op);
}

// sum_t abar[t] * m_t^AX * w[t - e_AX]: the derivative of a per-axis shift with
// respect to the shift velocity, d/du (N1(-u)) = D N1(-u) and d/du N1(u) = -D N1(u)
// with (D v)_m = m v_{m-1}, contracted with the adjoint.
template <int AX, typename R>
__device__ __forceinline__ R lowered_dot(const R (&abar)[27], const R (&w)[27])
{
    R acc = R(0);
    sfor<0, 27>([&](auto T) {
        constexpr int t = decltype(T)::value;
        constexpr int k = AX == 0 ? sa(t) : (AX == 1 ? sb(t) : sc(t));
        constexpr int st = AX == 0 ? 9 : (AX == 1 ? 3 : 1);
        if constexpr (k == 1) acc = fma(abar[t], w[t - st], acc);
        if constexpr (k == 2) acc = fma(R(2) * abar[t], w[t - st], acc);
    });
    return acc;
}

}  // namespace clbm

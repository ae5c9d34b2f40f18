// HIP kernels of the D3Q27 cascaded LBM for gfx950 (MI355X).
//
// Memory layout: a state is [27][P] in the storage type (structure of arrays,
// x fastest; plane stride P >= N, the first N entries of a plane used), so a
// wavefront of 64 lanes on 64 consecutive nodes reads and
// writes 64 consecutive elements of each population plane.  The step is a
// "pull" step: node x gathers population i from x - e_i of the previous
// post-collision state (Eq. (8) read backwards), collides in registers and
// writes its 27 post-collision values at x, so every store is aligned and
// coalesced and every value crosses HBM exactly once in each direction.
// Half-way bounce-back replaces a blocked pull by the node's own opposite
// population.  The work per node is ~550 flops against 2 x 27 values moved, so
// the kernel is bound by HBM bandwidth; nothing here is a dense contraction
// and no MFMA is used.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "node.hpp"

namespace clbm {

constexpr int kBlock = 256;

// ------------------------------------------------------------------ storage types
template <typename S>
struct Traits;
template <>
struct Traits<double> {
    using R = double;                   // arithmetic type
    static constexpr bool kDev = false; // stores f itself
};
template <>
struct Traits<float> {
    using R = float;
    static constexpr bool kDev = true;  // stores f - w
};
template <>
struct Traits<_Float16> {
    using R = float;
    static constexpr bool kDev = true;
};
template <>
struct Traits<__bf16> {
    using R = float;
    static constexpr bool kDev = true;
};

template <typename S>
__device__ __forceinline__ typename Traits<S>::R to_real(S v) { return static_cast<typename Traits<S>::R>(v); }

// Round a real (FP32 or FP64) to the storage type, nearest-even.
template <typename S, typename R>
__device__ __forceinline__ S to_store(R v)
{
    if constexpr (std::is_same<S, double>::value)
        return static_cast<double>(v);
    else
        return static_cast<S>(static_cast<float>(v));
}

// ------------------------------------------------------------------ geometry
// n / d for n < 2^31 by multiply-shift (Granlund-Montgomery with 31-bit
// numerators): m = floor(2^(31+l) / d) + 1, l = ceil(log2 d).
struct FastDiv {
    uint64_t mul;
    uint32_t shift;
    uint32_t d;
    __host__ void init(uint32_t d_)
    {
        d = d_;
        uint32_t l = 0;
        while ((1ull << l) < d_) ++l;
        shift = 31 + l;
        mul = ((1ull << shift) / d_) + 1;
    }
    __host__ __device__ __forceinline__ uint32_t div(uint32_t n) const
    {
        return static_cast<uint32_t>((static_cast<uint64_t>(n) * mul) >> shift);
    }
};

constexpr uint32_t kZGroup = 8;            // planes per group of the z-grouped node order
constexpr uint32_t kZGroupMinPlane = 98304;  // nodes per plane from which that order is used

struct Geom {
    uint32_t N, nx, ny, nz, nxy;
    uint32_t P;        // plane stride of state buffers in elements (>= N; padding breaks power-of-two strides)
    FastDiv dnx, dny;
    FastDiv dzg;       // rows of a whole z group, kZGroup * ny (zgroup_node)
    FastDiv dzr;       // planes of the last z group when nz is not a multiple of kZGroup (else 1)
    uint32_t zgroup;   // nonzero: kernels that read a link table visit nodes in z-grouped order
    int32_t wall[3];
    int32_t moving;    // bit f set when wall face f moves (0 = no moving wall)
    double wu[6][3];   // velocity of wall face (axis a, side s) at [2a + s]; side 1 lies beyond n_a - 1
};

// Pull sources of one node.  Index a = e + 1 per axis: xs[a] is the x of the node
// x - e (wrapped on periodic axes), ys/zs the row/plane offsets; v* says whether
// that neighbour exists (false beyond a wall).  Offsets stay in range even when
// the neighbour does not exist.
struct Nbr {
    uint32_t xs[3], ys[3], zs[3];
    bool vx[3], vy[3], vz[3];
};

__device__ __forceinline__ void axis_sources(uint32_t c, uint32_t n, int32_t wall, uint32_t (&s)[3], bool (&v)[3])
{
    // a = 0 (e = -1): source c + 1;  a = 1: c;  a = 2 (e = +1): source c - 1
    const bool top = (c + 1 == n), bot = (c == 0);
    s[0] = top ? 0u : c + 1;
    s[1] = c;
    s[2] = bot ? n - 1 : c - 1;
    v[0] = !(top && wall);
    v[1] = true;
    v[2] = !(bot && wall);
}

__device__ __forceinline__ void node_coords(const Geom &g, uint32_t n, uint32_t &x, uint32_t &y, uint32_t &z)
{
    const uint32_t yz = g.dnx.div(n);
    x = n - yz * g.nx;
    z = g.dny.div(yz);
    y = yz - z * g.ny;
}

__device__ __forceinline__ void neighbours_xyz(const Geom &g, uint32_t x, uint32_t y, uint32_t z, Nbr &nb)
{
    axis_sources(x, g.nx, g.wall[0], nb.xs, nb.vx);
    axis_sources(y, g.ny, g.wall[1], nb.ys, nb.vy);
    axis_sources(z, g.nz, g.wall[2], nb.zs, nb.vz);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        nb.ys[k] *= g.nx;
        nb.zs[k] *= g.nxy;
    }
}

__device__ __forceinline__ void neighbours(const Geom &g, uint32_t n, Nbr &nb)
{
    uint32_t x, y, z;
    node_coords(g, n, x, y, z);
    neighbours_xyz(g, x, y, z, nb);
}

// Is the link pulled by slot t open (neighbour x - e exists and is fluid)?  When
// REV, the link towards x + e instead.  Without solids the walls are tested from
// the coordinates; with solids the node's link word lm (see k_links) holds the
// answer for every slot, walls included.
template <int T, bool REV, bool LINKS>
__device__ __forceinline__ bool link_open(const Nbr &nb, uint32_t lm, uint32_t &off)
{
    constexpr int a = REV ? 2 - sa(T) : sa(T), b = REV ? 2 - sb(T) : sb(T), c = REV ? 2 - sc(T) : sc(T);
    off = nb.zs[c] + nb.ys[b] + nb.xs[a];
    if constexpr (LINKS)
        return (lm >> (REV ? 26 - T : T)) & 1u;
    else
        return nb.vx[a] && nb.vy[b] && nb.vz[c];
}

// Element at a 32-bit byte offset from a wavefront-uniform base.  Every
// population plane has its own base (kept in scalar registers), so each load or
// store needs one 32-bit per-lane offset instead of a 64-bit per-lane address.
// A plane therefore spans less than 4 GiB: N * sizeof(element) < 2^32.
template <typename T>
__device__ __forceinline__ T load_at(const T *__restrict__ base, uint32_t byte_off)
{
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + byte_off);
}
// Stores of whole state and adjoint planes are streaming: nothing reads them back
// before the next kernel, and a lattice is far larger than the caches.  They are
// issued non-temporal (measured 2-3% faster on the 512^3 FP32 step, up to 8% for
// FP64).  Loads stay ordinary: the x-shifted pulls of a wavefront share cache lines.
template <typename T>
__device__ __forceinline__ void store_at(T *__restrict__ base, uint32_t byte_off, T v)
{
    __builtin_nontemporal_store(v, reinterpret_cast<T *>(reinterpret_cast<char *>(base) + byte_off));
}

// Momentum exchange of moving walls for a blocked pull of slot T: the
// population that left along -e through the wall faces it crossed returns as
// slot T with + 2 w (e . u_w)/c_s^2, u_w the mean velocity of those faces (zero
// when the link is blocked by a solid node only).
template <int T, int Q, typename R>
__device__ __forceinline__ R wall_term(const Nbr &nb, const Geom &g)
{
    R ux = R(0), uy = R(0), uz = R(0);
    int cnt = 0;
    auto add = [&](int face) {
        ux += static_cast<R>(g.wu[face][0]);
        uy += static_cast<R>(g.wu[face][1]);
        uz += static_cast<R>(g.wu[face][2]);
        ++cnt;
    };
    // pulling slot index 0 (e = -1) reads x + 1: crosses the face beyond n - 1; index 2 the face below 0
    if constexpr (sa(T) != 1)
        if (!nb.vx[sa(T)]) add(0 + (sa(T) == 0 ? 1 : 0));
    if constexpr (sb(T) != 1)
        if (!nb.vy[sb(T)]) add(2 + (sb(T) == 0 ? 1 : 0));
    if constexpr (sc(T) != 1)
        if (!nb.vz[sc(T)]) add(4 + (sc(T) == 0 ? 1 : 0));
    if (cnt == 0) return R(0);
    const R eu = R(sa(T) - 1) * ux + R(sb(T) - 1) * uy + R(sc(T) - 1) * uz;
    const R mean = cnt == 1 ? R(1) : (cnt == 2 ? R(0.5) : R(1.0 / 3.0));  // 1 / faces crossed
    return R(6) * lattice_weight<Q, R>(T) * eu * mean;
}

// Does the node lie on a moving wall face (face 2 axis + side: side 0 below
// coordinate 0, side 1 beyond n - 1)?  Links of other nodes cross only resting
// faces, where the momentum term is zero and is not formed.
__device__ __forceinline__ bool on_moving_face(const Geom &g, const Nbr &nb)
{
    const uint32_t m = static_cast<uint32_t>(g.moving);
    return ((m & 1u) && !nb.vx[2]) || ((m & 2u) && !nb.vx[0]) || ((m & 4u) && !nb.vy[2]) ||
           ((m & 8u) && !nb.vy[0]) || ((m & 16u) && !nb.vz[2]) || ((m & 32u) && !nb.vz[0]);
}

template <typename S, bool CHECK, bool SOLID, bool REV, int Q, typename R>
__device__ __forceinline__ void gather_links(const S *__restrict__ buf, const Geom &g, uint32_t n, const Nbr &nb,
                                             uint32_t lm, R (&v)[27]);

// Gather of Eq. (8): v[t] = population of slot t arriving at node n, as a real
// (the stored value, deviation or not).  REV gathers along +e instead (adjoint).
// With walls or solids, a wavefront whose nodes all have their 26 links open
// (the common case) takes the unchecked path; only wavefronts touching a wall or
// a solid test every link.  Lattice Q (27 or 19): slots without a population
// (the D3Q19 corners) read nothing and hold 0.
template <int Q>
__host__ __device__ constexpr uint32_t all_links()
{
    uint32_t m = 0;
    for (int t = 0; t < 27; ++t)
        if (has_slot<Q>(t)) m |= 1u << t;
    return m;
}

template <typename S, bool CHECK, bool SOLID, bool REV, int Q = 27, typename R>
__device__ __forceinline__ void gather(const S *__restrict__ buf, const Geom &g, uint32_t n, const Nbr &nb,
                                       uint32_t lm, R (&v)[27])
{
    if constexpr (CHECK) {
        bool open;
        if constexpr (SOLID)
            open = lm == all_links<Q>();
        else
            open = nb.vx[0] && nb.vx[2] && nb.vy[0] && nb.vy[2] && nb.vz[0] && nb.vz[2];
        if (__all(open))
            gather_links<S, false, false, REV, Q>(buf, g, n, nb, lm, v);
        else
            gather_links<S, true, SOLID, REV, Q>(buf, g, n, nb, lm, v);
    } else {
        gather_links<S, false, false, REV, Q>(buf, g, n, nb, lm, v);
    }
}

template <typename S, bool CHECK, bool SOLID, bool REV, int Q, typename R>
__device__ __forceinline__ void gather_links(const S *__restrict__ buf, const Geom &g, uint32_t n, const Nbr &nb,
                                             uint32_t lm, R (&v)[27])
{
    // forward gathers read state buffers (plane stride P); reverse gathers read
    // adjoint buffers, which are dense [27][N]
    const size_t N = REV ? static_cast<size_t>(g.N) : static_cast<size_t>(g.P);
    constexpr uint32_t es = sizeof(S);
    const bool mf = !REV && CHECK && g.moving && on_moving_face(g, nb);
    sfor<0, 27>([&](auto TT) {
        constexpr int t = decltype(TT)::value;
        constexpr int i = pop_of_slot(t);
        const S *__restrict__ Pi = buf + static_cast<size_t>(i) * N;
        if constexpr (!has_slot<Q>(t)) {
            v[t] = R(0);
        } else if constexpr (t == 13) {
            v[t] = static_cast<R>(to_real(load_at(Pi, n * es)));
        } else {
            uint32_t off;
            const bool ok = link_open<t, REV, SOLID>(nb, lm, off);
            if constexpr (CHECK) {
                constexpr int ib = pop_of_slot(26 - t);
                S val;
                if (ok)
                    val = load_at(Pi, off * es);
                else
                    val = load_at(buf + static_cast<size_t>(ib) * N, n * es);
                v[t] = static_cast<R>(to_real(val));
                if constexpr (!REV)
                    if (mf && !ok) v[t] += wall_term<t, Q, R>(nb, g);
            } else {
                v[t] = static_cast<R>(to_real(load_at(Pi, off * es)));
            }
        }
    });
}

// Inverse of gather: write the value of slot t of node n where gather() reads it.
template <typename S, bool CHECK, bool SOLID, int Q, typename R>
__device__ __forceinline__ void scatter(S *__restrict__ buf, const Geom &g, uint32_t n, const Nbr &nb, uint32_t lm,
                                        const R (&v)[27])
{
    const size_t N = g.P;  // state buffer
    const bool mf = CHECK && g.moving && on_moving_face(g, nb);
    sfor<0, 27>([&](auto TT) {
        constexpr int t = decltype(TT)::value;
        constexpr int i = pop_of_slot(t);
        S *__restrict__ Pi = buf + static_cast<size_t>(i) * N;
        S val = to_store<S>(v[t]);
        if constexpr (!has_slot<Q>(t)) {
            // no population in this slot
        } else if constexpr (t == 13) {
            Pi[n] = val;
        } else {
            uint32_t off;
            const bool ok = link_open<t, false, SOLID>(nb, lm, off);
            if constexpr (CHECK) {
                constexpr int ib = pop_of_slot(26 - t);
                if (mf && !ok) val = to_store<S>(v[t] - wall_term<t, Q, R>(nb, g));
                S *p = ok ? (Pi + off) : (buf + static_cast<size_t>(ib) * N + n);
                *p = val;
            } else {
                Pi[off] = val;
            }
        }
    });
}

// Link table for lattices with solid nodes (and for walled lattices that take the
// fused two-step kernel; solid = NULL then): word n has bit t set when the pull of
// slot t into node n is open (the neighbour n - e exists and is fluid) and bit 13
// (the rest population) set for every fluid node; solid nodes get 0.  One
// coalesced 32-bit load per node then replaces 26 dependent mask loads.
template <int Q>
__global__ __launch_bounds__(kBlock) void k_links(Geom g, const uint8_t *__restrict__ solid, uint32_t *__restrict__ links)
{
    const uint32_t n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.N) return;
    Nbr nb;
    neighbours(g, n, nb);
    uint32_t m = 0;
    sfor<0, 27>([&](auto TT) {
        constexpr int t = decltype(TT)::value;
        uint32_t off;
        if (has_slot<Q>(t) && link_open<t, false, false>(nb, 0u, off) && (!solid || solid[off] == 0)) m |= 1u << t;
    });
    links[n] = solid && solid[n] ? 0u : (m | (1u << 13));
}

template <typename R>
struct Forcing {
    R F[3];   // uniform part
    R scale;  // multiplies the per-node field
};

// Raw per-node field values (zero without a field) and the force they give.
template <bool FIELD, typename R>
__device__ __forceinline__ void load_field(const R *__restrict__ field, uint32_t N, uint32_t n, R &fx, R &fy, R &fz)
{
    fx = fy = fz = R(0);
    if constexpr (FIELD) {
        const uint32_t off = n * static_cast<uint32_t>(sizeof(R));
        fx = load_at(field, off);
        fy = load_at(field + N, off);
        fz = load_at(field + 2 * static_cast<size_t>(N), off);
    }
}

template <bool FIELD, typename R>
__device__ __forceinline__ void force_from(const Forcing<R> &fo, R fx, R fy, R fz, R &Fx, R &Fy, R &Fz)
{
    Fx = fo.F[0];
    Fy = fo.F[1];
    Fz = fo.F[2];
    if constexpr (FIELD) {
        Fx = fma(fo.scale, fx, Fx);
        Fy = fma(fo.scale, fy, Fy);
        Fz = fma(fo.scale, fz, Fz);
    }
}

template <bool FIELD, typename R>
__device__ __forceinline__ void force_at(const Forcing<R> &fo, const R *__restrict__ field, uint32_t N, uint32_t n,
                                         R &Fx, R &Fy, R &Fz)
{
    R fx, fy, fz;
    load_field<FIELD>(field, N, n, fx, fy, fz);
    force_from<FIELD>(fo, fx, fy, fz, Fx, Fy, Fz);
}

// ------------------------------------------------------------------ XCD-aware block order
// MI355X dispatches consecutive workgroups round-robin over its 8 XCDs, each with
// its own L2.  Remapping block b so that XCD k processes the k-th contiguous
// eighth of the lattice keeps neighbouring tiles of a row on one XCD: the cache
// lines that the x-shifted pulls share between adjacent tiles are then fetched
// from HBM once instead of once per XCD.  The map is a bijection on [0, nb).
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nb)
{
    const uint32_t q = nb / 8, r = nb % 8, x = b % 8, k = b / 8;
    return x * q + (x < r ? x : r) + k;
}

// Node at position p of the z-grouped order of the kernels that read a link table
// (solid nodes): x fastest, then the planes of a group of kZGroup, then y, then the
// groups.  A fluid node next to a solid takes its own opposite population, from a
// cache line that the pulls of the row at (y, z) - e also read.  In row order the
// rows at z +- 1 are a whole plane of blocks apart; once a plane holds more nodes
// than the blocks resident on an XCD cover, those lines come from HBM twice (the
// adjoint read 292 B per node instead of about 245 on the 20%-solid duct).  In
// this order most such pairs of rows run within a few blocks of each other (255 B).
// Measured on 16 lattice shapes, the order is faster from about 100k nodes per
// plane (adjoint +4% to +11%, single step up to +8%) and slower below (up to -14%:
// there the row order already finds much of the reuse in L2, and the concurrent
// blocks of the z-grouped order spread over eight planes), hence kZGroupMinPlane.
__device__ __forceinline__ uint32_t zgroup_node(const Geom &g, uint32_t p)
{
    const uint32_t r = g.dnx.div(p), x = p - r * g.nx;
    const uint32_t grp = g.dzg.div(r), w = r - grp * (kZGroup * g.ny);
    uint32_t y, z;
    if ((grp + 1) * kZGroup <= g.nz) {
        y = w / kZGroup;
        z = grp * kZGroup + w % kZGroup;
    } else {
        y = g.dzr.div(w);
        z = grp * kZGroup + (w - y * g.dzr.d);
    }
    return x + g.nx * (y + g.ny * z);
}

// ------------------------------------------------------------------ forward step
// Collision models of the step kernels.
enum Collision : int {
    kCascaded = 0,       // Sec. II B, Eq. (5)
    kCascadedHigh1 = 1,  // the same when every rate above second order is one (collide_high1)
    kMrt = 2,            // raw-moment MRT with Guo forcing (Appendix B)
};

// Steps 1-3 of Sec. II B on one node's deviations d = f - w (in place, registers).
// Q = 19: the D3Q19 scheme of Appendix A on the same slots (corner slots hold 0
// on entry and exit).
template <int COLL = kCascaded, int Q = 27, typename R>
__device__ __forceinline__ void node_update(R (&v)[27], R Fx, R Fy, R Fz, const Rates<R> &rt)
{
    if constexpr (COLL == kMrt) {
        static_assert(Q == 27, "the MRT runs on D3Q27");
        collide_mrt(v, Fx, Fy, Fz, rt);
        return;
    }
    if constexpr (Q == 19) {
        static_assert(COLL == kCascaded, "D3Q19 uses the general collision");
        raw_moments(v);
        const R drho = v[slot(0, 0, 0)];
        const R inv_rho = R(1) / (R(1) + drho);
        const R ux = (v[slot(1, 0, 0)] + R(0.5) * Fx) * inv_rho;
        const R uy = (v[slot(0, 1, 0)] + R(0.5) * Fy) * inv_rho;
        const R uz = (v[slot(0, 0, 1)] + R(0.5) * Fz) * inv_rho;
        central_shift(v, ux, uy, uz);
        const AxisU<R> X(ux), Y(uy), Z(uz);
        collide(v, drho, X, Y, Z, Fx, Fy, Fz, rt);  // Eq. (A3), (A5), (A6) on the moments of Eq. (A2)
        reconstruct_q19(v, ux, uy, uz);
        return;
    }
    if constexpr (COLL == kCascadedHigh1) {
        R ux, uy, uz;
        collide_high1(v, Fx, Fy, Fz, rt, ux, uy, uz);
        reconstruct(v, ux, uy, uz);
        return;
    }
    raw_moments(v);  // Eq. (4), (14): T = M d
    const R drho = v[slot(0, 0, 0)];
    const R inv_rho = R(1) / (R(1) + drho);  // Eq. (9)
    const R ux = (v[slot(1, 0, 0)] + R(0.5) * Fx) * inv_rho;
    const R uy = (v[slot(0, 1, 0)] + R(0.5) * Fy) * inv_rho;
    const R uz = (v[slot(0, 0, 1)] + R(0.5) * Fz) * inv_rho;
    central_shift(v, ux, uy, uz);  // T~ = N(u) T
    const AxisU<R> X(ux), Y(uy), Z(uz);
    collide(v, drho, X, Y, Z, Fx, Fy, Fz, rt);  // Eq. (5)
    reconstruct(v, ux, uy, uz);                 // Eq. (7): N^-1 then M^-1
}

// One fused time step on one node per thread (Steps 1-4 of Sec. II B).
// A solid node reads nothing but still runs the arithmetic on the rest state and
// stores its (never read) entries, so that every wavefront writes whole cache
// lines: lanes that skipped their stores would leave partially written lines,
// which cost far more memory time than the extra bytes.
template <typename S, bool CHECK, bool SOLID, bool FIELD, int COLL, int Q>
__device__ __forceinline__ void step_node(uint32_t n, const S *__restrict__ src, S *__restrict__ dst, const Geom &g,
                                          const uint32_t *__restrict__ links,
                                          const typename Traits<S>::R *__restrict__ field,
                                          const Forcing<typename Traits<S>::R> &fo,
                                          const Rates<typename Traits<S>::R> &rt)
{
    using R = typename Traits<S>::R;
    if (n >= g.N) return;
    uint32_t lm = 0;
    if constexpr (SOLID) lm = links[n];
    Nbr nb;
    neighbours(g, n, nb);
    R v[27];
    // FP32/FP16/BF16: raised wavefront priority until the pulls are consumed, as in the fused kernel
    // (+2% to +5% on these storage types; FP64, whose node update is twice as long, lost 4% with it)
    constexpr bool kPrio = !std::is_same<S, double>::value;
    if constexpr (kPrio) __builtin_amdgcn_s_setprio(3);
    if (!SOLID || lm != 0u) {
        gather<S, CHECK, SOLID, false, Q>(src, g, n, nb, lm, v);
        if constexpr (!Traits<S>::kDev)
            sfor<0, 27>([&](auto T) { v[decltype(T)::value] -= lattice_weight<Q, R>(decltype(T)::value); });
    } else {
        sfor<0, 27>([&](auto T) { v[decltype(T)::value] = R(0); });
    }

    R Fx, Fy, Fz;
    force_at<FIELD>(fo, field, g.N, n, Fx, Fy, Fz);
    if constexpr (kPrio) __builtin_amdgcn_s_setprio(0);
    node_update<COLL, Q>(v, Fx, Fy, Fz, rt);

    const uint32_t nb_off = n * static_cast<uint32_t>(sizeof(S));
    sfor<0, 27>([&](auto TT) {
        constexpr int t = decltype(TT)::value;
        if constexpr (has_slot<Q>(t)) {
            R val = v[t];
            if constexpr (!Traits<S>::kDev) val += lattice_weight<Q, R>(t);
            store_at(dst + static_cast<size_t>(pop_of_slot(t)) * g.P, nb_off, to_store<S>(val));
        }
    });
}

template <typename S, bool CHECK, bool SOLID, bool FIELD, int COLL, int Q>
__global__ __launch_bounds__(kBlock) void k_step(const S *__restrict__ src, S *__restrict__ dst, Geom g,
                                                 const uint32_t *__restrict__ links,
                                                 const typename Traits<S>::R *__restrict__ field,
                                                 Forcing<typename Traits<S>::R> fo, Rates<typename Traits<S>::R> rt)
{
    const uint32_t p = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    step_node<S, CHECK, SOLID, FIELD, COLL, Q>(SOLID && g.zgroup && p < g.N ? zgroup_node(g, p) : p, src, dst, g,
                                               links, field, fo, rt);
}

// ------------------------------------------------------------------ two fused steps (temporal blocking)
// Two time steps per launch on FP32 and FP64 lattices: D3Q27 with the cascaded
// collision or the MRT of Appendix B, and D3Q19 (Q = 19: only the 19 population
// planes are read and written, the corner slots hold 0).  A block owns a 32 x 12
// tile of (x, y) columns (32 x 16 for periodic FP64 lattices with the cascaded
// collision, see t2_rows) and marches along a chunk of z planes.
// For each plane it first runs step t -> t+1 on the tile plus a one-node halo
// (34 x 14 nodes, pulling from HBM), keeping the results in LDS, and then step
// t+1 -> t+2 on the tile plane below, pulling those results from LDS and
// writing to HBM.  The intermediate state never leaves the chip, so HBM moves
// about 1.24 x 27 reads (the halo) and 27 writes per node for two updates
// instead of 2 x (27 + 27).  Intermediate values are rounded to the storage
// type exactly as a stored state would be, so the result is bitwise that of
// two single steps.
//
// LDS: step t+2 at plane z pulls the e_z = -1 populations from plane z+1, e_z = 0
// from plane z and e_z = +1 from plane z-1 of the intermediate state.  Each
// thread keeps its halo node's e_z = 0 group for one plane iteration and its
// e_z = +1 group for two in registers and writes a group to LDS only in the
// iteration that pulls it, so LDS holds just three groups of 9 x 476 values
// (51 KB per block in FP32; FP64 doubles it to 103 KB, one block per CU).  The tile height was chosen by measurement (heights 6 to 16
// on 512^3, 640x320x320 and 128^3 lattices; 12 was fastest on all three).
//
// With solid nodes or walls (SOLID: the link table holds every node's open
// links) the bounce-back of Eq. (8) in step t+2 takes the node's own opposite
// population from step t+1 (plus the momentum of a moving wall).  Each tile
// node is then stepped in t+2 by the thread that stepped it in t+1 (threads 0
// to 383 take the tile, wavefronts 6 and 7 the halo ring), whose registers hold the
// node's e_z = +1 group and link word; the e_z = 0 group of plane z is in LDS,
// and the e_z = -1 groups alternate between two LDS slots by plane parity so
// that plane z's stays readable while plane z+1's is written (68.5 KB per block in
// FP32, 137 KB in FP64).
// Population i's slot (inverse of pop_of_slot).
__host__ __device__ constexpr int slot_of_pop(int i)
{
    for (int t = 0; t < 27; ++t)
        if (pop_of_slot(t) == i) return t;
    return -1;
}
constexpr bool slot_of_pop_inverts()
{
    for (int t = 0; t < 27; ++t)
        if (slot_of_pop(pop_of_slot(t)) != t) return false;
    return true;
}
static_assert(slot_of_pop_inverts(), "pop_of_slot is a bijection of the 27 slots and slot_of_pop its inverse");

// Address of population plane i + 1 from that of plane i, for loops over the planes in
// increasing order inside the fused kernel's plane loop.  Left to itself the compiler
// keeps all 27 source and 27 destination plane addresses live across that loop (108
// scalar registers): they do not fit beside the rest of the kernel's uniform state, so
// they are spilled to vector lanes and each reload costs two vector instructions on
// every load and store.  The empty asm makes the running byte offset opaque, so each
// address is formed by scalar adds where it is used.  The first-step loads use it in
// both variants; the link-table variant also stores this way, while the periodic
// variant, whose 27 destination addresses fit once the loads no longer hold 27 more,
// keeps its stores in slot order.  (The offset, not the address,
// goes through the asm: an address derived from the kernel argument by arithmetic
// keeps its global address space, and the accesses keep their scalar-base form.)
template <typename T>
__device__ __forceinline__ T *next_plane(T *base, uint64_t &off, uint64_t stride_bytes)
{
    using B = typename std::conditional<std::is_const<T>::value, const char, char>::type;
    off += stride_bytes;
    asm volatile("" : "+s"(off));
    return reinterpret_cast<T *>(reinterpret_cast<B *>(base) + off);
}

// The value a stored state holds in slot t for the post-collision deviation d: storage types that
// hold deviations round d, FP64 storage holds f = d + w_t (as step_node stores it).
template <typename S, int Q, int t, typename R>
__device__ __forceinline__ R stored_value(R d)
{
    if constexpr (!Traits<S>::kDev) d += lattice_weight<Q, R>(t);
    return static_cast<R>(to_store<S>(d));
}

// The deviation d = f - w_t the node update takes, from a value as a state holds it.
template <typename S, typename R, int Q>
__device__ __forceinline__ void to_deviations(R (&v)[27])
{
    if constexpr (!Traits<S>::kDev)
        sfor<0, 27>([&](auto T) { v[decltype(T)::value] -= lattice_weight<Q, R>(decltype(T)::value); });
}

constexpr int kT2X = 32, kT2HX = kT2X + 2;  // tile columns, and with the halo
// Rows of the tile.  FP32 arithmetic: 12 (two 8-wave blocks per CU; 6 to 16 rows were measured and
// 12 was fastest).  FP64: the ring of doubles leaves room for one block per CU, and 16 rows (10 waves,
// 132 KB of LDS, at most 168 registers) ran the cascaded collision 7-16% faster than 12 rows, and 8
// rows (two 6-wave blocks per CU) 5-15% slower; the MRT, whose FP64 update spills at 168
// registers, keeps 12 rows and 256 registers (16 rows were 13% slower), and so does the link-table
// variant, whose four LDS groups of doubles fill 137 KB at 12 rows.
__host__ __device__ constexpr int t2_rows(bool fp64, int coll, bool links)
{
    return fp64 && coll != kMrt && !links ? 16 : 12;
}
template <typename R, int COLL, bool SOLID>
struct T2Tile {
    static constexpr int Y = t2_rows(sizeof(R) == 8, COLL, SOLID);
    static constexpr int HY = Y + 2, H = kT2HX * HY;  // halo tile: 476 nodes at 12 rows, 612 at 16
    static constexpr int Block = (H + 63) / 64 * 64;  // 512 threads at 12 rows, 640 at 16
    // waves per SIMD the register budget must allow: 4 (128 registers) for FP32, 2 (256) for the
    // one 8-wave FP64 block, 3 (168) for the one 10-wave FP64 block
    static constexpr int WavesPerEU = sizeof(R) == 4 ? 4 : (Block > 512 ? 3 : 2);
};
// Dynamic LDS requested with each launch of the variant without a link table: it keeps that
// kernel at two blocks per CU.  Its 51 KB ring alone would let a third block in whenever
// the kernel needs 80 VGPRs or fewer, and three blocks per CU ran the 512^3 lattice 27%
// slower.  (The link-table variant's 68.5 KB ring already admits only two.)
constexpr unsigned kT2PadLds = 4096;

struct T2Geom {
    uint32_t tiles_x, tiles_y, zchunk;
};

__device__ __forceinline__ uint32_t wrap_coord(int c, uint32_t n)
{
    int r = c % static_cast<int>(n);
    return static_cast<uint32_t>(r < 0 ? r + static_cast<int>(n) : r);
}

// (the waves-per-EU bound sets the register budget: 128 for FP32 arithmetic; FP64 arithmetic,
// whose values take two registers each, runs one block per CU with 168 or 256)
template <typename S, bool FIELD, int COLL, bool SOLID, int Q = 27>
__global__ __launch_bounds__((T2Tile<typename Traits<S>::R, COLL, SOLID>::Block)) __attribute__((
    amdgpu_waves_per_eu(T2Tile<typename Traits<S>::R, COLL, SOLID>::WavesPerEU))) void k_step2(
    const S *__restrict__ src, S *__restrict__ dst, Geom g, T2Geom tg, const uint32_t *__restrict__ links,
    const typename Traits<S>::R *__restrict__ field, Forcing<typename Traits<S>::R> fo,
    Rates<typename Traits<S>::R> rt)
{
    using R = typename Traits<S>::R;
    using Tile = T2Tile<R, COLL, SOLID>;
    static constexpr int kT2Y = Tile::Y, kT2HY = Tile::HY, kT2H = Tile::H, kT2Block = Tile::Block;
    // [0]: e_z = -1 group of plane z+1, [1]: e_z = 0 group of plane z, [2]: e_z = +1 group of plane z-1;
    // with SOLID, [0] and [3] hold the e_z = -1 groups of even and odd planes.  The ring holds the
    // arithmetic type, which represents every storable value exactly.
    __shared__ R ring[SOLID ? 4 : 3][9][kT2H];
    auto zm = [](int p) { return SOLID && (p & 1) ? 3 : 0; };

    const uint32_t b = xcd_block(blockIdx.x, gridDim.x);
    const uint32_t tx = b % tg.tiles_x, rest = b / tg.tiles_x;
    const uint32_t ty = rest % tg.tiles_y, zc = rest / tg.tiles_y;
    const int x0 = static_cast<int>(tx) * kT2X, y0 = static_cast<int>(ty) * kT2Y;
    const int z0 = static_cast<int>(zc * tg.zchunk);
    const int z1 = min(z0 + static_cast<int>(tg.zchunk), static_cast<int>(g.nz));
    const int tid = threadIdx.x;

    // Halo position (hx, hy) of this thread in step t+1 and its LDS index hs = hy * kT2HX + hx.
    // Without solids: row-major (hs = tid); step t+2 of tile node (cx, cy) runs on thread
    // cy * kT2X + cx.  With solids, step t+2 of a tile node must run on the thread that stepped
    // it in t+1 (its registers hold the node's own values), so threads 0 ... 383 (wavefronts 0-5)
    // take the tile nodes row by row.  The 92 halo-ring nodes go to wavefronts 6 and 7, each
    // taking one whole halo row (34 nodes, corners included; coalesced) and the 12 column nodes
    // of one side.  A column node is alone in its row, so each of its loads touches a cache line
    // of its own; split over two wavefronts, those lines cost each wavefront's loads half as much,
    // and the wavefronts that wait for the slowest at the plane barrier wait less.
    int hx = 0, hy = 0;
    bool ha;
    if constexpr (SOLID) {
        constexpr int kCore = kT2X * kT2Y;
        static_assert(kCore % 64 == 0 && kCore + 128 == kT2Block && kT2HX + kT2Y <= 64,
                      "tile rows fill wavefronts 0-5 and the halo ring fits wavefronts 6 and 7");
        ha = true;
        if (tid < kCore) {
            hx = 1 + tid % kT2X;
            hy = 1 + tid / kT2X;
        } else {
            const int side = (tid - kCore) >> 6, l = (tid - kCore) & 63;
            if (l < kT2HX) {
                hx = l;
                hy = side ? kT2HY - 1 : 0;
            } else if (l < kT2HX + kT2Y) {
                hx = side ? kT2HX - 1 : 0;
                hy = 1 + (l - kT2HX);
            } else {
                ha = false;  // 18 idle lanes in each of the two halo wavefronts
            }
        }
    } else {
        hx = tid % kT2HX;
        hy = tid / kT2HX;
        ha = tid < kT2H;
    }
    const int hs = hy * kT2HX + hx;
    const uint32_t gx = wrap_coord(x0 - 1 + hx, g.nx), gy = wrap_coord(y0 - 1 + hy, g.ny);
    const int cx = tid % kT2X, cy = tid / kT2X;
    const bool ca = tid < kT2X * kT2Y && x0 + cx < static_cast<int>(g.nx) && y0 + cy < static_cast<int>(g.ny);

    const uint64_t plane_bytes = static_cast<uint64_t>(g.P) * sizeof(S);
    // groups of the halo node's intermediate values kept in registers until the plane that pulls
    // them: e_z = 0 of plane p, e_z = +1 of planes p - 1 and p (p: the last plane computed)
    R keep0[9], keep2a[9], keep2b[9];
    uint32_t lm_a = 0, lm_b = 0;  // SOLID: the halo node's link words in planes p - 1 and p
    // SOLID: the link word of the next plane, loaded one plane ahead.  The checked pulls need it
    // for their addresses, so loading it with them would put a second HBM round trip on the path
    // of every plane.
    uint32_t lm_next = 0;
    if constexpr (SOLID)
        if (ha) lm_next = links[gx + g.nx * (gy + g.ny * wrap_coord(z0 - 1, g.nz))];

    // The first step's wavefronts run at raised priority until their 27 pulls are consumed: the
    // arbiter then issues their loads ahead of the other block's arithmetic, so more memory is in
    // flight while the SIMDs compute (measured +10% on the 512^3 headline, +5% on the porous duct).
    auto first_step = [&](int p) {
        if (!ha) return;
        __builtin_amdgcn_s_setprio(3);
        const uint32_t pz = wrap_coord(p, g.nz);
        const uint32_t n = gx + g.nx * (gy + g.ny * pz);
        Nbr nb;
        neighbours_xyz(g, gx, gy, pz, nb);
        constexpr uint32_t es = sizeof(S);
        R v[27];
        if constexpr (SOLID) {
            const uint32_t lm = lm_next;
            lm_next = links[gx + g.nx * (gy + g.ny * wrap_coord(p + 1, g.nz))];
            lm_a = lm_b;
            lm_b = lm;
            if (lm == 0u) {
                sfor<0, 27>([&](auto T) { v[decltype(T)::value] = R(0); });  // solid: the rest state, as step_node
            } else if (__all(lm == all_links<Q>())) {
                const S *__restrict__ pl = src;  // plane i, planes in increasing order
                uint64_t po = 0;
                sfor<0, 27>([&](auto II) {
                    constexpr int i = decltype(II)::value, t = slot_of_pop(i);
                    if constexpr (i < Q) {  // D3Q19: populations 0-18 (the corners come last in Eq. (1))
                        uint32_t off;
                        link_open<t, false, false>(nb, 0u, off);
                        v[t] = to_real(load_at(pl, off * es));
                        if constexpr (i < Q - 1) pl = next_plane(src, po, plane_bytes);
                    } else {
                        v[t] = R(0);
                    }
                });
                to_deviations<S, R, Q>(v);
            } else {
                // the gather of Eq. (8) with its checks, planes in increasing order: a blocked
                // link takes the node's own opposite population (plane ib), whose address is an
                // opaque multiple of the plane stride, formed in scalar registers where it is used
                const bool mf = g.moving && on_moving_face(g, nb);
                const S *__restrict__ pl = src;
                uint64_t po = 0;
                sfor<0, 27>([&](auto II) {
                    constexpr int i = decltype(II)::value, t = slot_of_pop(i);
                    if constexpr (i >= Q) {
                        v[t] = R(0);
                    } else if constexpr (t == 13) {
                        v[t] = to_real(load_at(pl, n * es));
                    } else {
                        constexpr int ib = pop_of_slot(26 - t);
                        uint32_t off;
                        const bool ok = link_open<t, false, true>(nb, lm, off);
                        uint64_t pb = plane_bytes;
                        asm volatile("" : "+s"(pb));
                        const S *__restrict__ own =
                            reinterpret_cast<const S *>(reinterpret_cast<const char *>(src) + pb * ib);
                        const S val = ok ? load_at(pl, off * es) : load_at(own, n * es);
                        v[t] = to_real(val);
                        if (mf && !ok) v[t] += wall_term<t, Q, R>(nb, g);
                    }
                    if constexpr (i < Q - 1) pl = next_plane(src, po, plane_bytes);
                });
                to_deviations<S, R, Q>(v);
            }
        } else {
            const S *__restrict__ pl = src;  // plane i, planes in increasing order
            uint64_t po = 0;
            sfor<0, 27>([&](auto II) {
                constexpr int i = decltype(II)::value, t = slot_of_pop(i);
                if constexpr (i < Q) {
                    uint32_t off;
                    link_open<t, false, false>(nb, 0u, off);
                    v[t] = to_real(load_at(pl, off * es));
                    if constexpr (i < Q - 1) pl = next_plane(src, po, plane_bytes);
                } else {
                    v[t] = R(0);
                }
            });
            to_deviations<S, R, Q>(v);
        }
        R Fx, Fy, Fz;
        force_at<FIELD>(fo, field, g.N, n, Fx, Fy, Fz);
        __builtin_amdgcn_s_setprio(0);
        node_update<COLL, Q>(v, Fx, Fy, Fz, rt);
        const int r0 = zm(p);
        sfor<0, 9>([&](auto J) {
            constexpr int j = decltype(J)::value;  // j = 3 a + b; slot 3 j + c with c = e_z + 1
            ring[r0][j][hs] = stored_value<S, Q, 3 * j + 0>(v[3 * j + 0]);  // the value a stored state would hold
            keep2a[j] = keep2b[j];
            keep0[j] = stored_value<S, Q, 3 * j + 1>(v[3 * j + 1]);
            keep2b[j] = stored_value<S, Q, 3 * j + 2>(v[3 * j + 2]);
        });
    };

    // Without solids, the force-field values of the second step are loaded one plane ahead, so
    // that the node update does not wait for them (the first step's loads carry its own).  The
    // link-table variant has no registers to spare for them.
    constexpr bool kFieldAhead = FIELD && !SOLID;
    auto tile_node = [&](int z) {
        return static_cast<uint32_t>(x0 + cx) +
               g.nx * (static_cast<uint32_t>(y0 + cy) + g.ny * wrap_coord(z, g.nz));
    };
    R fnx = R(0), fny = R(0), fnz = R(0);
    if constexpr (kFieldAhead)
        if (ca) load_field<FIELD>(field, g.N, tile_node(z0), fnx, fny, fnz);

    auto second_step = [&](int z) {
        if (!ca) return;
        const uint32_t zz = wrap_coord(z, g.nz);
        // with solids this thread stepped the same node in t+1: (gx, gy) and hs are the tile node's
        const uint32_t n = SOLID ? gx + g.nx * (gy + g.ny * zz)
                                 : static_cast<uint32_t>(x0 + cx) + g.nx * (static_cast<uint32_t>(y0 + cy) + g.ny * zz);
        const int hn = SOLID ? hs : (cy + 1) * kT2HX + (cx + 1);  // LDS index of the tile node
        R v[27];
        // slot t pulls from the halo position of x - e; index into the ring viewed as one array
        const R *rf = &ring[0][0][0];
        const int rz = zm(z + 1);
        auto pulled_at = [&](auto TT) -> int {
            constexpr int t = decltype(TT)::value;
            constexpr int a = sa(t), bb = sb(t), c = sc(t), j = 3 * a + bb;
            return ((c == 0 ? rz : c) * 9 + j) * kT2H + hn + (1 - bb) * kT2HX + (1 - a);
        };
        // the pulled value of slot t (D3Q19: the corner slots hold no population and stay 0)
        auto pull = [&](auto TT) -> R {
            constexpr int t = decltype(TT)::value;
            if constexpr (has_slot<Q>(t))
                return rf[pulled_at(TT)];
            else
                return R(0);
        };
        if constexpr (SOLID) {
            const uint32_t lm = lm_a;
            if (lm == 0u) {
                sfor<0, 27>([&](auto T) { v[decltype(T)::value] = R(0); });
            } else if (__all(lm == all_links<Q>())) {
                sfor<0, 27>([&](auto TT) { v[decltype(TT)::value] = pull(TT); });
                to_deviations<S, R, Q>(v);
            } else {
                // a blocked link returns the node's own opposite population of step t+1 (Eq. (8)),
                // plus the momentum of a moving wall as in gather()
                const int ro = zm(z);
                Nbr nb;
                bool mf = false;
                if (g.moving) {
                    neighbours_xyz(g, gx, gy, zz, nb);
                    mf = on_moving_face(g, nb);
                }
                sfor<0, 27>([&](auto TT) {
                    constexpr int t = decltype(TT)::value;
                    constexpr int jo = 8 - (3 * sa(t) + sb(t)), co = 2 - sc(t);
                    const R nbv = pull(TT);
                    if constexpr (t == 13 || !has_slot<Q>(t)) {
                        v[t] = nbv;
                    } else {
                        R own;
                        if constexpr (co == 2)
                            own = keep2a[jo];
                        else
                            own = rf[((co == 0 ? ro : 1) * 9 + jo) * kT2H + hn];
                        const bool open = (lm >> t) & 1u;
                        v[t] = open ? nbv : own;
                        if (mf && !open) v[t] += wall_term<t, Q, R>(nb, g);
                    }
                });
                to_deviations<S, R, Q>(v);
            }
        } else {
            sfor<0, 27>([&](auto TT) { v[decltype(TT)::value] = pull(TT); });
            to_deviations<S, R, Q>(v);
        }
        R Fx, Fy, Fz;
        if constexpr (kFieldAhead) {
            force_from<FIELD>(fo, fnx, fny, fnz, Fx, Fy, Fz);
            load_field<FIELD>(field, g.N, tile_node(z + 1), fnx, fny, fnz);
        } else {
            force_at<FIELD>(fo, field, g.N, n, Fx, Fy, Fz);
        }
        node_update<COLL, Q>(v, Fx, Fy, Fz, rt);
        const uint32_t nb_off = n * static_cast<uint32_t>(sizeof(S));
        if constexpr (SOLID) {
            // the link-table variant holds too many uniform values to keep the 27 destination
            // plane addresses as well: stores in plane order with the running offset
            S *__restrict__ pl = dst;
            uint64_t po = 0;
            sfor<0, Q>([&](auto II) {
                constexpr int i = decltype(II)::value, t = slot_of_pop(i);
                if constexpr (Traits<S>::kDev)
                    store_at(pl, nb_off, to_store<S>(v[t]));
                else
                    store_at(pl, nb_off, to_store<S>(v[t] + lattice_weight<Q, R>(t)));
                if constexpr (i < Q - 1) pl = next_plane(dst, po, plane_bytes);
            });
        } else {
            sfor<0, 27>([&](auto TT) {
                constexpr int t = decltype(TT)::value;
                if constexpr (has_slot<Q>(t)) {
                    R val = v[t];
                    if constexpr (!Traits<S>::kDev) val += lattice_weight<Q, R>(t);
                    store_at(dst + static_cast<size_t>(pop_of_slot(t)) * g.P, nb_off, to_store<S>(val));
                }
            });
        }
    };

    sfor<0, 9>([&](auto J) { keep2b[decltype(J)::value] = R(0); });
    first_step(z0 - 1);  // keep2b <- e_z = +1 group of plane z0 - 1
    first_step(z0);      // keep0 <- e_z = 0 of z0, keep2a <- +1 of z0 - 1, keep2b <- +1 of z0
    for (int z = z0; z < z1; ++z) {
        __syncthreads();  // the previous plane's pulls from the ring are done
        if (ha)
            sfor<0, 9>([&](auto J) {
                constexpr int j = decltype(J)::value;
                ring[1][j][hs] = keep0[j];   // e_z = 0 of plane z
                ring[2][j][hs] = keep2a[j];  // e_z = +1 of plane z - 1
            });
        first_step(z + 1);  // ring[zm(z + 1)] <- e_z = -1 of plane z + 1
        __syncthreads();    // the three groups of second_step(z) are in the ring
        second_step(z);
    }
}

// ------------------------------------------------------------------ block reductions (FP64, fixed order)
template <int NC>
__device__ __forceinline__ void block_reduce_store(double (&acc)[NC], double *__restrict__ out)
{
    __shared__ double red[kBlock / 64][NC];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        double x = acc[c];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
        if (lane == 0) red[wv][c] = x;
    }
    __syncthreads();
    if (threadIdx.x < NC) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) s += red[w][threadIdx.x];
        out[threadIdx.x] = s;
    }
}

// Sum partials[b * stride + c] over b < nblocks for c = blockIdx.x; out[c] = (acc ? out[c] : 0) + sum.
__global__ __launch_bounds__(kBlock) void k_reduce(const double *__restrict__ partials, int nblocks, int stride,
                                                   double *__restrict__ out, int accumulate)
{
    const int c = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += kBlock) s += partials[static_cast<size_t>(b) * stride + c];
    double acc[1] = {s};
    __shared__ double res[1];
    block_reduce_store<1>(acc, res);
    __syncthreads();
    if (threadIdx.x == 0) out[c] = (accumulate ? out[c] : 0.0) + res[0];
}

// First stage for long partial tables: block b sums rows b*kBlock ... b*kBlock+kBlock-1
// of partials[row][NC] (fixed order) into out[b][NC].
template <int NC>
__global__ __launch_bounds__(kBlock) void k_fold(const double *__restrict__ partials, int nrows,
                                                 double *__restrict__ out)
{
    const int r = blockIdx.x * kBlock + threadIdx.x;
    double acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = r < nrows ? partials[static_cast<size_t>(r) * NC + c] : 0.0;
    block_reduce_store<NC>(acc, out + static_cast<size_t>(blockIdx.x) * NC);
}

// ------------------------------------------------------------------ macroscopic fields (Eq. (9))
constexpr int kMomComp = 5;  // mass, momentum x/y/z, count of bad nodes

template <typename S, bool CHECK, bool SOLID, bool FIELD, int Q>
__global__ __launch_bounds__(kBlock) void k_moments(const S *__restrict__ src, Geom g,
                                                    const uint32_t *__restrict__ links,
                                                    const typename Traits<S>::R *__restrict__ field,
                                                    Forcing<typename Traits<S>::R> fo, double *__restrict__ rho_out,
                                                    double *__restrict__ u_out, double *__restrict__ partials)
{
    using R = typename Traits<S>::R;
    double acc[kMomComp] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (uint32_t n = blockIdx.x * kBlock + threadIdx.x; n < g.N; n += gridDim.x * kBlock) {
        const uint32_t lm = SOLID ? links[n] : 0u;
        if (SOLID && lm == 0u) {
            if (rho_out) rho_out[n] = 0.0;
            if (u_out) u_out[n] = u_out[g.N + n] = u_out[2 * static_cast<size_t>(g.N) + n] = 0.0;
            continue;
        }
        Nbr nb;
        neighbours(g, n, nb);
        double v[27];
        gather<S, CHECK, SOLID, false, Q>(src, g, n, nb, lm, v);
        if constexpr (!Traits<S>::kDev)
            sfor<0, 27>([&](auto T) { v[decltype(T)::value] -= lattice_weight<Q, double>(decltype(T)::value); });
        raw_moments(v);
        R Fx, Fy, Fz;
        force_at<FIELD>(fo, field, g.N, n, Fx, Fy, Fz);
        const double rho = 1.0 + v[slot(0, 0, 0)];
        const double mx = v[slot(1, 0, 0)] + 0.5 * static_cast<double>(Fx);
        const double my = v[slot(0, 1, 0)] + 0.5 * static_cast<double>(Fy);
        const double mz = v[slot(0, 0, 1)] + 0.5 * static_cast<double>(Fz);
        const double ux = mx / rho, uy = my / rho, uz = mz / rho;
        const bool bad = !(rho > 0.0) || !isfinite(rho) || !isfinite(ux) || !isfinite(uy) || !isfinite(uz);
        if (rho_out) rho_out[n] = rho;
        if (u_out) {
            u_out[n] = ux;
            u_out[g.N + n] = uy;
            u_out[2 * static_cast<size_t>(g.N) + n] = uz;
        }
        acc[0] += rho;
        acc[1] += mx;
        acc[2] += my;
        acc[3] += mz;
        acc[4] += bad ? 1.0 : 0.0;
    }
    block_reduce_store<kMomComp>(acc, partials + static_cast<size_t>(blockIdx.x) * kMomComp);
}

// ------------------------------------------------------------------ populations in/out, initial state
template <typename S, bool CHECK, bool SOLID, int Q>
__global__ __launch_bounds__(kBlock) void k_get_populations(const S *__restrict__ src, Geom g,
                                                            const uint32_t *__restrict__ links,
                                                            double *__restrict__ f)
{
    const uint32_t n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.N) return;
    const uint32_t lm = SOLID ? links[n] : 0u;
    if (SOLID && lm == 0u) {
        for (int i = 0; i < Q; ++i) f[static_cast<size_t>(i) * g.N + n] = 0.0;
        return;
    }
    Nbr nb;
    neighbours(g, n, nb);
    double v[27];
    gather<S, CHECK, SOLID, false, Q>(src, g, n, nb, lm, v);
    sfor<0, 27>([&](auto TT) {
        constexpr int t = decltype(TT)::value;
        if constexpr (has_slot<Q>(t)) {
            double val = v[t];
            if constexpr (Traits<S>::kDev) val += lattice_weight<Q, double>(t);
            f[static_cast<size_t>(pop_of_slot(t)) * g.N + n] = val;
        }
    });
}

// Pre-collision populations of `count` listed nodes: out[i][k] for node nodes[k].
template <typename S, bool CHECK, bool SOLID, int Q>
__global__ __launch_bounds__(kBlock) void k_sample_populations(const S *__restrict__ src, Geom g,
                                                               const uint32_t *__restrict__ links,
                                                               const int32_t *__restrict__ nodes, uint32_t count,
                                                               double *__restrict__ out)
{
    const uint32_t k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= count) return;
    const int32_t id = nodes[k];
    const bool valid = id >= 0 && static_cast<uint32_t>(id) < g.N;
    const uint32_t n = valid ? static_cast<uint32_t>(id) : 0u;
    const uint32_t lm = SOLID ? links[n] : 0u;
    if (!valid || (SOLID && lm == 0u)) {
        for (int i = 0; i < Q; ++i) out[static_cast<size_t>(i) * count + k] = valid ? 0.0 : NAN;
        return;
    }
    Nbr nb;
    neighbours(g, n, nb);
    double v[27];
    gather<S, CHECK, SOLID, false, Q>(src, g, n, nb, lm, v);
    sfor<0, 27>([&](auto TT) {
        constexpr int t = decltype(TT)::value;
        if constexpr (has_slot<Q>(t)) {
            double val = v[t];
            if constexpr (Traits<S>::kDev) val += lattice_weight<Q, double>(t);
            out[static_cast<size_t>(pop_of_slot(t)) * count + k] = val;
        }
    });
}

template <typename S, bool CHECK, bool SOLID, int Q>
__global__ __launch_bounds__(kBlock) void k_set_populations(const double *__restrict__ f, Geom g,
                                                            const uint32_t *__restrict__ links, S *__restrict__ dst)
{
    const uint32_t n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.N) return;
    const uint32_t lm = SOLID ? links[n] : 0u;
    if (SOLID && lm == 0u) return;
    Nbr nb;
    neighbours(g, n, nb);
    double v[27];
    sfor<0, 27>([&](auto TT) {
        constexpr int t = decltype(TT)::value;
        if constexpr (has_slot<Q>(t)) {
            double val = f[static_cast<size_t>(pop_of_slot(t)) * g.N + n];
            if constexpr (Traits<S>::kDev) val -= lattice_weight<Q, double>(t);
            v[t] = val;
        } else {
            v[t] = 0.0;
        }
    });
    scatter<S, CHECK, SOLID, Q>(dst, g, n, nb, lm, v);
}

// f = f_eq(rho0, u0): the generalized equilibrium (NM)^-1 T_eq, computed in FP64
// as the reconstruction of T_eq - N(u) M w; DISCRETE (the MRT of Appendix B):
// the discrete equilibrium f_D^eq of Sec. II B.
template <typename S, bool CHECK, bool SOLID, int Q, bool DISCRETE>
__global__ __launch_bounds__(kBlock) void k_init(S *__restrict__ dst, Geom g, const uint32_t *__restrict__ links,
                                                 const double *__restrict__ rho0, const double *__restrict__ u0)
{
    const uint32_t n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.N) return;
    const uint32_t lm = SOLID ? links[n] : 0u;
    if (SOLID && lm == 0u) return;
    Nbr nb;
    neighbours(g, n, nb);
    const double drho = rho0 ? rho0[n] - 1.0 : 0.0;
    const double ux = u0 ? u0[n] : 0.0;
    const double uy = u0 ? u0[g.N + n] : 0.0;
    const double uz = u0 ? u0[2 * static_cast<size_t>(g.N) + n] : 0.0;
    const AxisU<double> X(ux), Y(uy), Z(uz);
    double v[27];
    if constexpr (DISCRETE) {
        static_assert(Q == 27, "the discrete equilibrium is the D3Q27 one");
        discrete_equilibrium_dev(v, drho, ux, uy, uz);
    } else {
        equilibrium_moments(v, drho, X, Y, Z);
        if constexpr (Q == 19)
            reconstruct_q19(v, ux, uy, uz);
        else
            reconstruct(v, ux, uy, uz);
    }
    if constexpr (!Traits<S>::kDev)
        sfor<0, 27>([&](auto T) { v[decltype(T)::value] += lattice_weight<Q, double>(decltype(T)::value); });
    scatter<S, CHECK, SOLID, Q>(dst, g, n, nb, lm, v);
}

// ------------------------------------------------------------------ adjoint
// Rates whose adjoint is accumulated: s2 ... s6 (indices 2..9); s0 and s1 act on
// conserved moments and have zero derivative.
constexpr int kAdjRates = 8;

// One adjoint step on one node per thread (one thread per node, no grid-stride
// loop: a loop around this body keeps loop-invariant values in VGPRs and halves
// the occupancy).  Recomputes the forward
// moments from the state at t, gathers lambda(t+1) along +e (the transpose of
// the pull), applies the transposed per-node Jacobian and writes lambda(t).
//
// Per-axis shifts satisfy N1(-u) = exp(u D) and N1(u) = exp(-u D) with the
// lowering operator (D v)_m = m v_{m-1}, which commutes with both.  Hence the
// velocity derivatives of the two shifts, contracted with the adjoint, are
//   from N(-u):  abar~*^T D_a T~*,     from N(u):  -abar~^T D_a T~,
// in terms of the central moments before (T~) and after (T~*) the collision and
// their adjoints.  Only T~ and one adjoint vector are kept live; T~* is re-formed
// slot by slot from T~.
template <typename S, bool CHECK, bool SOLID, bool FIELD>
__device__ __forceinline__ void adjoint_nodes(const S *__restrict__ state, const Geom &g,
                                              const uint32_t *__restrict__ links,
                                              const typename Traits<S>::R *__restrict__ field,
                                              const Forcing<typename Traits<S>::R> &fo,
                                              const Rates<typename Traits<S>::R> &rt,
                                              const typename Traits<S>::R *__restrict__ lam_next,
                                              typename Traits<S>::R *__restrict__ lam_out,
                                              typename Traits<S>::R *__restrict__ dJdF, double *__restrict__ partials)
{
    using R = typename Traits<S>::R;
    constexpr R cs2 = R(1.0 / 3.0), cs4 = R(1.0 / 9.0);
    // this node's dJ/ds terms, summed over its moments in the arithmetic type; the sums over nodes are FP64
    R gsr[kAdjRates] = {};
    // XCD-aware order, as the step kernels: the +e shifted gathers of neighbouring blocks then share an L2
    // (z-grouped on large planes with solids, as k_step)
    const uint32_t p = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    const uint32_t n = SOLID && g.zgroup && p < g.N ? zgroup_node(g, p) : p;
    if (n < g.N) {
        // A solid node reads no state or adjoint: with zero inputs every output below is
        // exactly zero (lambda = 0, no force or rate contribution), and its stores keep
        // the wavefront's cache lines whole.
        uint32_t lm = 0;
        if constexpr (SOLID) lm = links[n];
        const bool fluid = !SOLID || lm != 0u;
        // accumulated force gradient of this node, loaded up front with the other operands
        R gFx = R(0), gFy = R(0), gFz = R(0);
        if (dJdF) {
            gFx = dJdF[n];
            gFy = dJdF[g.N + n];
            gFz = dJdF[2 * static_cast<size_t>(g.N) + n];
        }
        Nbr nb;
        neighbours(g, n, nb);
        // ---- forward recomputation: T~ (full central moments) at this node
        R tt[27];
        if (fluid) {
            gather<S, CHECK, SOLID, false>(state, g, n, nb, lm, tt);
            if constexpr (!Traits<S>::kDev)
                sfor<0, 27>([&](auto T) { tt[decltype(T)::value] -= weight_of_slot<R>(decltype(T)::value); });
        } else {
            sfor<0, 27>([&](auto T) { tt[decltype(T)::value] = R(0); });
        }
        raw_moments(tt);
        const R rho = R(1) + tt[slot(0, 0, 0)];
        const R inv_rho = R(1) / rho;
        R Fx, Fy, Fz;
        force_at<FIELD>(fo, field, g.N, n, Fx, Fy, Fz);
        const R ux = (tt[slot(1, 0, 0)] + R(0.5) * Fx) * inv_rho;
        const R uy = (tt[slot(0, 1, 0)] + R(0.5) * Fy) * inv_rho;
        const R uz = (tt[slot(0, 0, 1)] + R(0.5) * Fz) * inv_rho;
        central_shift(tt, ux, uy, uz);
        {
            const AxisU<R> X(ux), Y(uy), Z(uz);
            sfor<0, 27>([&](auto T) {
                constexpr int t = decltype(T)::value;
                tt[t] += cw_term<sa(t), sb(t), sc(t)>(X, Y, Z);
            });
        }
        // non-equilibrium part of the normal-stress block (Eq. (13)), shared by T~* and the rates
        constexpr int ix = slot(2, 0, 0), iy = slot(0, 2, 0), iz = slot(0, 0, 2);
        const R rx = fma(rho, cs2, -tt[ix]), ry = fma(rho, cs2, -tt[iy]), rz = fma(rho, cs2, -tt[iz]);
        const R rsum = rx + ry + rz;

        // ---- adjoint of f*: gather lambda(t+1) along +e, then through M^-1 and N(-u)
        R a[27];
        if (fluid)
            gather<R, CHECK, SOLID, true>(lam_next, g, n, nb, lm, a);
        else
            sfor<0, 27>([&](auto T) { a[decltype(T)::value] = R(0); });
        reconstruct_raw_T(a);
        unshift_T(a, ux, uy, uz);  // a = adjoint of T~*

        // u-derivative of N(-u): sum_b T~*(b) * m * a(b + e_axis) over the slots b below each axis
        R ubx = R(0), uby = R(0), ubz = R(0);
        sfor<0, 27>([&](auto T) {
            constexpr int b = decltype(T)::value;
            constexpr int m = sa(b), nn = sb(b), p = sc(b);
            if constexpr (m < 2 || nn < 2 || p < 2) {
                constexpr int ones = (m == 1) + (nn == 1) + (p == 1);
                constexpr int order = m + nn + p;
                R ts;  // post-collision central moment T~*(b), Eq. (5)
                if constexpr (order == 0) {
                    ts = rho;
                } else if constexpr (order == 1) {
                    ts = R(0.5) * (m == 1 ? Fx : (nn == 1 ? Fy : Fz));
                } else if constexpr (order == 2 && ones == 0) {
                    const R r = b == ix ? rx : (b == iy ? ry : rz);
                    ts = tt[b] + fma(rt.s[R_S2], r, rt.sm * rsum);
                } else {
                    constexpr int k = rate_of(m, nn, p);
                    constexpr R E = R(e_of(m) * e_of(nn) * e_of(p));
                    R r = -tt[b];
                    if constexpr (ones == 0) r = fma(rho, E, r);
                    ts = fma(rt.s[k], r, tt[b]);
                    if constexpr (ones == 1) {
                        constexpr R cf = order == 3 ? cs2 : cs4;
                        const R Fa = m == 1 ? Fx : (nn == 1 ? Fy : Fz);
                        ts = fma(rt.hs[k] * cf, Fa, ts);
                    }
                }
                if constexpr (m < 2) ubx = fma(R(m + 1) * a[b + 9], ts, ubx);
                if constexpr (nn < 2) uby = fma(R(nn + 1) * a[b + 3], ts, uby);
                if constexpr (p < 2) ubz = fma(R(p + 1) * a[b + 1], ts, ubz);
            }
        });

        // ---- collision backward: a <- (I - S) a on non-conserved slots, conserved slots feed rho and F
        R rhob = a[slot(0, 0, 0)];
        R Fbx = R(0.5) * a[slot(1, 0, 0)], Fby = R(0.5) * a[slot(0, 1, 0)], Fbz = R(0.5) * a[slot(0, 0, 1)];
        a[slot(0, 0, 0)] = R(0);
        a[slot(1, 0, 0)] = R(0);
        a[slot(0, 1, 0)] = R(0);
        a[slot(0, 0, 1)] = R(0);
        sfor<0, 27>([&](auto T) {
            constexpr int t = decltype(T)::value;
            constexpr int m = sa(t), nn = sb(t), p = sc(t);
            constexpr int ones = (m == 1) + (nn == 1) + (p == 1);
            constexpr int order = m + nn + p;
            if constexpr (order >= 2 && !(order == 2 && ones == 0)) {
                constexpr int k = rate_of(m, nn, p);
                constexpr R E = R(e_of(m) * e_of(nn) * e_of(p));
                const R y = a[t];
                R r = -tt[t];  // rho E - T~ - C/2
                if constexpr (ones == 0) r = fma(rho, E, r);
                if constexpr (ones == 1) {
                    constexpr R cf = order == 3 ? cs2 : cs4;
                    const R Fa = m == 1 ? Fx : (nn == 1 ? Fy : Fz);
                    r = fma(R(-0.5) * cf, Fa, r);
                    const R gF = rt.hs[k] * cf * y;
                    if constexpr (m == 1) Fbx += gF;
                    else if constexpr (nn == 1) Fby += gF;
                    else Fbz += gF;
                }
                gsr[k - 2] = fma(y, r, gsr[k - 2]);
                if constexpr (ones == 0) rhob = fma(rt.s[k] * E, y, rhob);
                a[t] = fma(-rt.s[k], y, y);
            }
        });
        {
            const R yx = a[ix], yy = a[iy], yz = a[iz];
            const R ysum = yx + yy + yz;
            const R tr = rt.sm * ysum;
            const R sx = fma(rt.s[R_S2], yx, tr), sy = fma(rt.s[R_S2], yy, tr), sz = fma(rt.s[R_S2], yz, tr);
            a[ix] = yx - sx;
            a[iy] = yy - sy;
            a[iz] = yz - sz;
            rhob = fma(cs2, sx + sy + sz, rhob);
            const R third = ysum * rsum * R(1.0 / 3.0);
            gsr[R_S2 - 2] += fma(yx, rx, fma(yy, ry, yz * rz)) - third;
            gsr[R_S2B - 2] += third;
        }
        // u-derivative of N(u), then back through N(u) and M
        ubx -= lowered_dot<0>(a, tt);
        uby -= lowered_dot<1>(a, tt);
        ubz -= lowered_dot<2>(a, tt);
        shift_T(a, ux, uy, uz);
        // u = (j + F/2) / rho
        a[slot(1, 0, 0)] += ubx * inv_rho;
        a[slot(0, 1, 0)] += uby * inv_rho;
        a[slot(0, 0, 1)] += ubz * inv_rho;
        Fbx = fma(R(0.5) * inv_rho, ubx, Fbx);
        Fby = fma(R(0.5) * inv_rho, uby, Fby);
        Fbz = fma(R(0.5) * inv_rho, ubz, Fbz);
        rhob -= (ubx * ux + uby * uy + ubz * uz) * inv_rho;
        a[slot(0, 0, 0)] += rhob;
        raw_moments_T(a);  // lambda(t) = M^T a

        const uint32_t nb_off = n * static_cast<uint32_t>(sizeof(R));
        sfor<0, 27>([&](auto TT) {
            constexpr int t = decltype(TT)::value;
            store_at(lam_out + static_cast<size_t>(pop_of_slot(t)) * g.N, nb_off, a[t]);
        });
        if (dJdF) {
            dJdF[n] = gFx + Fbx;
            dJdF[g.N + n] = gFy + Fby;
            dJdF[2 * static_cast<size_t>(g.N) + n] = gFz + Fbz;
        }
    }
    double gs[kAdjRates];
#pragma unroll
    for (int k = 0; k < kAdjRates; ++k) gs[k] = static_cast<double>(gsr[k]);
    block_reduce_store<kAdjRates>(gs, partials + static_cast<size_t>(blockIdx.x) * kAdjRates);
}

template <typename S, bool CHECK, bool SOLID, bool FIELD>
__global__ __launch_bounds__(kBlock) void k_adjoint(const S *__restrict__ state, Geom g,
                                                    const uint32_t *__restrict__ links,
                                                    const typename Traits<S>::R *__restrict__ field,
                                                    Forcing<typename Traits<S>::R> fo, Rates<typename Traits<S>::R> rt,
                                                    const typename Traits<S>::R *__restrict__ lam_next,
                                                    typename Traits<S>::R *__restrict__ lam_out,
                                                    typename Traits<S>::R *__restrict__ dJdF,
                                                    double *__restrict__ partials)
{
    adjoint_nodes<S, CHECK, SOLID, FIELD>(state, g, links, field, fo, rt, lam_next, lam_out, dJdF, partials);
}

// Loss J = 1/2 sum_fluid |u - u_t|^2 and its seed lambda = dJ/df; adds dJ/dF (direct).
// Solid nodes read no state and contribute nothing, but store zeros (whole lines).
template <typename S, bool CHECK, bool SOLID, bool FIELD>
__global__ __launch_bounds__(kBlock) void k_loss(const S *__restrict__ state, Geom g,
                                                 const uint32_t *__restrict__ links,
                                                 const typename Traits<S>::R *__restrict__ field,
                                                 Forcing<typename Traits<S>::R> fo,
                                                 const typename Traits<S>::R *__restrict__ u_target,
                                                 typename Traits<S>::R *__restrict__ lam_out,
                                                 typename Traits<S>::R *__restrict__ dJdF, double *__restrict__ partials)
{
    using R = typename Traits<S>::R;
    double acc[1] = {0.0};
    for (uint32_t n = blockIdx.x * kBlock + threadIdx.x; n < g.N; n += gridDim.x * kBlock) {
        uint32_t lm = 0;
        if constexpr (SOLID) lm = links[n];
        const bool fluid = !SOLID || lm != 0u;
        Nbr nb;
        neighbours(g, n, nb);
        R v[27];
        if (fluid) {
            gather<S, CHECK, SOLID, false>(state, g, n, nb, lm, v);
            if constexpr (!Traits<S>::kDev)
                sfor<0, 27>([&](auto T) { v[decltype(T)::value] -= weight_of_slot<R>(decltype(T)::value); });
        } else {
            sfor<0, 27>([&](auto T) { v[decltype(T)::value] = R(0); });
        }
        raw_moments(v);
        R Fx, Fy, Fz;
        force_at<FIELD>(fo, field, g.N, n, Fx, Fy, Fz);
        const R inv_rho = R(1) / (R(1) + v[slot(0, 0, 0)]);
        const R ux = (v[slot(1, 0, 0)] + R(0.5) * Fx) * inv_rho;
        const R uy = (v[slot(0, 1, 0)] + R(0.5) * Fy) * inv_rho;
        const R uz = (v[slot(0, 0, 1)] + R(0.5) * Fz) * inv_rho;
        const R dx = fluid ? ux - u_target[n] : R(0);
        const R dy = fluid ? uy - u_target[g.N + n] : R(0);
        const R dz = fluid ? uz - u_target[2 * static_cast<size_t>(g.N) + n] : R(0);
        acc[0] += 0.5 * (static_cast<double>(dx) * dx + static_cast<double>(dy) * dy + static_cast<double>(dz) * dz);
        // dJ/df_i = sum_a d_a (e_ia - u_a) / rho
        const R bx = dx * inv_rho, by = dy * inv_rho, bz = dz * inv_rho;
        const R base = -(bx * ux + by * uy + bz * uz);
        sfor<0, 27>([&](auto TT) {
            constexpr int t = decltype(TT)::value;
            R val = base;
            if constexpr (sa(t) == 2) val += bx;
            if constexpr (sa(t) == 0) val -= bx;
            if constexpr (sb(t) == 2) val += by;
            if constexpr (sb(t) == 0) val -= by;
            if constexpr (sc(t) == 2) val += bz;
            if constexpr (sc(t) == 0) val -= bz;
            lam_out[static_cast<size_t>(pop_of_slot(t)) * g.N + n] = val;
        });
        if (dJdF) {
            dJdF[n] += R(0.5) * bx;
            dJdF[g.N + n] += R(0.5) * by;
            dJdF[2 * static_cast<size_t>(g.N) + n] += R(0.5) * bz;
        }
    }
    block_reduce_store<1>(acc, partials + blockIdx.x);
}

// ------------------------------------------------------------------ plain copy (checkpoints)
__global__ __launch_bounds__(kBlock) void k_copy16(const uint4 *__restrict__ src, uint4 *__restrict__ dst, size_t n16)
{
    for (size_t k = blockIdx.x * static_cast<size_t>(kBlock) + threadIdx.x; k < n16;
         k += static_cast<size_t>(gridDim.x) * kBlock)
        dst[k] = src[k];
}

__global__ void k_copy_tail(const uint8_t *__restrict__ src, uint8_t *__restrict__ dst, size_t n)
{
    const size_t k = threadIdx.x;
    if (k < n) dst[k] = src[k];
}

}  // namespace clbm

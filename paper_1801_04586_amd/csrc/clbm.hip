// Host side of the C ABI declared in include/clbm.h: argument validation,
// launch geometry, variant dispatch and FP64 reductions for the D3Q27 (and
// D3Q19) cascaded LBM kernels in kernels.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/clbm.h"
#include "host_logic.hpp"
#include "kernels.hpp"

using namespace clbm;

namespace {

constexpr int kMaxBlocks = 2048;   // grid of the grid-stride kernels (8 blocks per CU)
constexpr int kPartialStride = 8;  // doubles per block in the partials buffer (>= kMomComp, kAdjRates)

thread_local char g_err[clbm_host::kErrLen] = "no error";

// Static scratch of clbm_adjoint_step_noalloc: the per-block dJ/ds partial sums of k_adjoint (one row
// of kAdjRates doubles per kBlock nodes) and the rows k_fold reduces them to.  Sized for lattices of up
// to 2^25 nodes: 131072 + 512 rows, 8.03 MiB on each device the library runs on, held until the process
// ends.  Host code never uses the symbol itself as an address: each device's address comes from
// hipGetSymbolAddress (scratch_address) and is kept with the context.
constexpr size_t kNoallocMaxNodes = size_t(1) << 25;
constexpr size_t kNoallocRows = kNoallocMaxNodes / kBlock;
constexpr size_t kNoallocFoldedRows = kNoallocRows / kBlock;
static_assert(kNoallocRows % kBlock == 0, "folded rows cover the partial rows exactly");
constexpr int kMaxDevices = 64;

std::mutex g_scratch_mutex;
double *g_scratch_ptr[kMaxDevices] = {};

}  // namespace

static __device__ __align__(256) double scratch[(kNoallocRows + kNoallocFoldedRows) * kAdjRates];

struct clbm_ctx {
    clbm_desc d;
    hipStream_t stream;
    Geom geom;
    size_t nodes;
    double *partials;  // [partial_blocks + folded rows][kPartialStride]
    double *scal;      // [16] reduction results
    uint32_t *links;   // [N] link table (k_links) when the lattice has solid nodes, else NULL
    uint32_t options;  // CLBM_OPT_* flags
    int num_cu;        // compute units of the device
    int device;        // device the context was created on
    double *scratch;   // that device's address of the static scratch (clbm_adjoint_step_noalloc)
    int t2_slots[2][2][2][3][2];  // resident blocks of the fused kernel, by (FP64, links, force field, collision, D3Q19); 0 = unknown
    char err[clbm_host::kErrLen];
};

namespace {

int fail(clbm_ctx *c, int code, const char *fmt, const char *arg = "")
{
    char *dst = c ? c->err : g_err;
    std::snprintf(dst, clbm_host::kErrLen, fmt, arg);
    return code;
}

int hip_fail(clbm_ctx *c, hipError_t e, const char *what)
{
    char *dst = c ? c->err : g_err;
    std::snprintf(dst, clbm_host::kErrLen, "%s: %s", what, hipGetErrorString(e));
    return CLBM_EHIP;
}

int check_launch(clbm_ctx *c, const char *what)
{
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? CLBM_OK : hip_fail(c, e, what);
}

bool aligned(const void *p) { return clbm_host::aligned16(p); }

int validate_rates(clbm_ctx *c, const double *s) { return clbm_host::validate_rates(c ? c->err : g_err, s); }

int validate_desc(const clbm_desc *d) { return clbm_host::validate_desc(d, g_err); }

using clbm_host::store_size;
int lattice_q(const clbm_desc &d) { return d.lattice == CLBM_D3Q19 ? 19 : 27; }

template <typename R>
Rates<R> make_rates(const double *s)
{
    Rates<R> r;
    for (int k = 0; k < 10; ++k) {
        r.s[k] = static_cast<R>(s[k]);
        r.hs[k] = static_cast<R>(1.0 - 0.5 * s[k]);
    }
    r.sm = static_cast<R>((s[R_S2B] - s[R_S2]) / 3.0);
    return r;
}

template <typename R>
Forcing<R> make_forcing(const clbm_desc &d)
{
    Forcing<R> f;
    for (int a = 0; a < 3; ++a) f.F[a] = static_cast<R>(d.force_uniform[a]);
    f.scale = static_cast<R>(d.force_scale);
    return f;
}

// Compile-time variant of the kernels: storage type, which boundary/force code is
// needed, and the lattice (27 or 19 velocities).
template <typename S, bool C, bool So, bool Fi, int Qv>
struct V {
    using Store = S;
    using R = typename Traits<S>::R;
    static constexpr bool check = C, solid = So, field = Fi;
    static constexpr int q = Qv;
};

template <typename S, int Qv, typename F>
int dispatch_flags(const clbm_ctx *c, F &&f)
{
    const bool solid = c->links != nullptr;
    const bool check = solid || c->d.wall[0] || c->d.wall[1] || c->d.wall[2];
    const bool field = c->d.force != nullptr;
    if (solid) return field ? f(V<S, true, true, true, Qv>{}) : f(V<S, true, true, false, Qv>{});
    if (check) return field ? f(V<S, true, false, true, Qv>{}) : f(V<S, true, false, false, Qv>{});
    return field ? f(V<S, false, false, true, Qv>{}) : f(V<S, false, false, false, Qv>{});
}

template <int Qv, typename F>
int dispatch_storage(const clbm_ctx *c, F &&f)
{
    switch (c->d.storage) {
    case CLBM_F64: return dispatch_flags<double, Qv>(c, f);
    case CLBM_F32: return dispatch_flags<float, Qv>(c, f);
    case CLBM_F16: return dispatch_flags<_Float16, Qv>(c, f);
    default: return dispatch_flags<__bf16, Qv>(c, f);
    }
}

template <typename F>
int dispatch(const clbm_ctx *c, F &&f)
{
    return c->d.lattice == CLBM_D3Q19 ? dispatch_storage<19>(c, f) : dispatch_storage<27>(c, f);
}

// The adjoint and the loss exist for the D3Q27 cascaded scheme only.
template <typename F>
int dispatch_d3q27(clbm_ctx *c, F &&f)
{
    if (c->d.lattice != CLBM_D3Q27) return fail(c, CLBM_EINVAL, "the adjoint needs the D3Q27 lattice");
    if (c->d.collision != CLBM_CASCADED) return fail(c, CLBM_EINVAL, "the adjoint needs the cascaded collision");
    return dispatch_storage<27>(c, f);
}

unsigned node_blocks(const clbm_ctx *c) { return static_cast<unsigned>((c->nodes + kBlock - 1) / kBlock); }

// Device address of the static scratch on device dev (current), looked up once per device.
hipError_t scratch_address(int dev, double **out)
{
    *out = nullptr;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

// Blocks whose partial sums the context's scratch holds: the grid-stride kernels
// use at most kMaxBlocks; the adjoint and loss kernels (D3Q27 cascaded lattices
// only) run one block per kBlock nodes.
size_t partial_blocks(const clbm_ctx *c)
{
    const bool adjoint = c->d.lattice == CLBM_D3Q27 && c->d.collision == CLBM_CASCADED;
    const size_t b = adjoint ? node_blocks(c) : 0;
    return b > static_cast<size_t>(kMaxBlocks) ? b : static_cast<size_t>(kMaxBlocks);
}
unsigned stride_blocks(const clbm_ctx *c)
{
    const unsigned b = node_blocks(c);
    return b < static_cast<unsigned>(kMaxBlocks) ? b : static_cast<unsigned>(kMaxBlocks);
}

// Every rate above second order (s3, s3b, s4, s4b, s5, s6) equal to one: the
// collision then needs no moments beyond second order (collide_high1).
bool high_rates_one(const clbm_ctx *c)
{
    for (int k = 4; k < 10; ++k)
        if (c->d.s[k] != 1.0) return false;
    return true;
}

// Collision variant of the step kernels for a context.
int collision_of(const clbm_ctx *c)
{
    if (c->d.collision == CLBM_MRT) return kMrt;
    return c->d.lattice == CLBM_D3Q27 && high_rates_one(c) ? kCascadedHigh1 : kCascaded;
}

// Rows of the fused kernel's tile on this lattice (D3Q19 takes the general cascaded collision).
int fused_rows(const clbm_ctx *c)
{
    return t2_rows(c->d.storage == CLBM_F64, c->d.lattice == CLBM_D3Q19 ? kCascaded : collision_of(c),
                   c->links != nullptr);
}

int launch_step(clbm_ctx *c, const void *src, void *dst)
{
    const int coll = collision_of(c);
    return dispatch(c, [&](auto v) {
        using Vt = decltype(v);
        using S = typename Vt::Store;
        using R = typename Vt::R;
        auto go = [&](auto cc) {
            constexpr int C = decltype(cc)::value;
            hipLaunchKernelGGL((k_step<S, Vt::check, Vt::solid, Vt::field, C, Vt::q>), dim3(node_blocks(c)),
                               dim3(kBlock), 0, c->stream, static_cast<const S *>(src), static_cast<S *>(dst), c->geom,
                               c->links, static_cast<const R *>(c->d.force), make_forcing<R>(c->d),
                               make_rates<R>(c->d.s));
            return check_launch(c, "step kernel launch");
        };
        // D3Q19 takes the general cascaded collision only
        if constexpr (Vt::q == 27) {
            if (coll == kMrt) return go(std::integral_constant<int, kMrt>{});
            if (coll == kCascadedHigh1) return go(std::integral_constant<int, kCascadedHigh1>{});
        }
        return go(std::integral_constant<int, kCascaded>{});
    });
}

// Two fused steps per launch apply to lattices with FP32 or FP64 storage (D3Q27
// with the cascaded collision or the MRT, D3Q19 with the cascaded collision),
// either periodic or with a link table (solid nodes or walls, moving or not); in
// FP64 one block runs per compute unit, its LDS groups of doubles filling
// 103-137 KB.  For 16-bit storage (half the bytes of FP32) the single-step kernel
// is faster, the fused kernel's cost per step being set by its arithmetic and
// barriers rather than by memory.
bool fused_kind(const clbm_desc &d)
{
    return d.storage == CLBM_F32 || d.storage == CLBM_F64;
}

// A lattice too small to give the fused kernel two blocks per compute unit (tile
// columns x z chunks of at least 8 planes) runs single steps by default, whose
// 256-node blocks fill the device (64^3: 96 fused blocks, 25.9 us per step
// against 13.8 us for single steps).
bool fused_pairs(const clbm_ctx *c)
{
    if ((c->options & CLBM_OPT_SINGLE_STEP) || !fused_kind(c->d)) return false;
    if (!c->links && (c->d.wall[0] || c->d.wall[1] || c->d.wall[2])) return false;
    if (c->options & CLBM_OPT_FUSED_PAIRS) return true;
    const int rows = fused_rows(c);
    const uint64_t tiles = static_cast<uint64_t>((c->geom.nx + kT2X - 1) / kT2X) * ((c->geom.ny + rows - 1) / rows);
    const uint64_t chunks = c->geom.nz / 8 > 1 ? c->geom.nz / 8 : 1;
    return tiles * chunks >= 2 * static_cast<uint64_t>(c->num_cu);
}

using clbm_host::fused_chunks;

int launch_step2(clbm_ctx *c, const void *src, void *dst)
{
    const int coll = collision_of(c);
    auto go = [&](auto tag, auto field_tag, auto solid_tag) {
        using S = decltype(tag);
        using R = typename Traits<S>::R;
        constexpr bool FIELD = decltype(field_tag)::value;
        constexpr bool SOLID = decltype(solid_tag)::value;
        auto launch = [&](auto cc, auto qq) {
            constexpr int C = decltype(cc)::value;
            constexpr int Q = decltype(qq)::value;
            using Tile = T2Tile<R, C, SOLID>;
            T2Geom tg;
            tg.tiles_x = (c->geom.nx + kT2X - 1) / kT2X;
            tg.tiles_y = (c->geom.ny + Tile::Y - 1) / Tile::Y;
            const uint32_t tiles = tg.tiles_x * tg.tiles_y;
            constexpr unsigned dyn_lds = SOLID ? 0u : kT2PadLds;
            int &slots = c->t2_slots[sizeof(S) == 8 ? 1 : 0][SOLID ? 1 : 0][FIELD ? 1 : 0][C][Q == 19 ? 1 : 0];
            if (slots == 0) {
                int per_cu = 0;
                if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_step2<S, FIELD, C, SOLID, Q>, Tile::Block,
                                                                 dyn_lds) != hipSuccess ||
                    per_cu < 1)
                    per_cu = 1;
                slots = per_cu * c->num_cu;
            }
            const uint32_t nchunks_req = fused_chunks(tiles, c->geom.nz, static_cast<uint32_t>(slots));
            tg.zchunk = (c->geom.nz + nchunks_req - 1) / nchunks_req;
            const uint32_t nchunks = (c->geom.nz + tg.zchunk - 1) / tg.zchunk;
            const unsigned blocks = tiles * nchunks;
            hipLaunchKernelGGL((k_step2<S, FIELD, C, SOLID, Q>), dim3(blocks), dim3(Tile::Block), dyn_lds, c->stream,
                               static_cast<const S *>(src), static_cast<S *>(dst), c->geom, tg, c->links,
                               static_cast<const R *>(c->d.force), make_forcing<R>(c->d), make_rates<R>(c->d.s));
            return check_launch(c, "fused two-step kernel launch");
        };
        using Q27 = std::integral_constant<int, 27>;
        // D3Q19 (Appendix A) takes the general cascaded collision only
        if (c->d.lattice == CLBM_D3Q19)
            return launch(std::integral_constant<int, kCascaded>{}, std::integral_constant<int, 19>{});
        if (coll == kCascadedHigh1) return launch(std::integral_constant<int, kCascadedHigh1>{}, Q27{});
        if (coll == kMrt) return launch(std::integral_constant<int, kMrt>{}, Q27{});
        return launch(std::integral_constant<int, kCascaded>{}, Q27{});
    };
    if (c->d.storage == CLBM_F64) {
        if (c->links)
            return c->d.force != nullptr ? go(double{}, std::true_type{}, std::true_type{})
                                         : go(double{}, std::false_type{}, std::true_type{});
        return c->d.force != nullptr ? go(double{}, std::true_type{}, std::false_type{})
                                     : go(double{}, std::false_type{}, std::false_type{});
    }
    if (c->d.storage != CLBM_F32) return fail(c, CLBM_EINVAL, "fused step pairs take FP32 or FP64 storage");
    if (c->links)
        return c->d.force != nullptr ? go(float{}, std::true_type{}, std::true_type{})
                                     : go(float{}, std::false_type{}, std::true_type{});
    return c->d.force != nullptr ? go(float{}, std::true_type{}, std::false_type{})
                                 : go(float{}, std::false_type{}, std::false_type{});
}

}  // namespace

extern "C" {

int clbm_abi_version(void) { return CLBM_ABI_VERSION; }

int64_t clbm_default_plane_stride(int32_t nx, int32_t ny, int32_t nz, int32_t storage)
{
    return clbm_host::default_plane_stride(nx, ny, nz, storage);
}

const char *clbm_strerror(int status) { return clbm_host::status_string(status); }

const char *clbm_last_error(const clbm_ctx *ctx) { return ctx ? ctx->err : g_err; }

int clbm_create(clbm_ctx **out, const clbm_desc *desc, void *stream)
{
    if (!out) return fail(nullptr, CLBM_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate_desc(desc);
    if (rc) return rc;
    clbm_ctx *c = new (std::nothrow) clbm_ctx();
    if (!c) return fail(nullptr, CLBM_EINVAL, "out of host memory");
    c->d = *desc;
    c->stream = static_cast<hipStream_t>(stream);
    c->nodes = static_cast<size_t>(desc->nx) * desc->ny * desc->nz;
    Geom &g = c->geom;
    g.nx = desc->nx;
    g.ny = desc->ny;
    g.nz = desc->nz;
    g.nxy = g.nx * g.ny;
    g.N = static_cast<uint32_t>(c->nodes);
    g.P = desc->plane_stride ? static_cast<uint32_t>(desc->plane_stride) : g.N;
    g.dnx.init(g.nx);
    g.dny.init(g.ny);
    // (a group wider than 2^31 rows means nz < kZGroup: one partial group, any divisor above the row count will do)
    g.dzg.init(static_cast<uint32_t>(std::min<uint64_t>(uint64_t(kZGroup) * g.ny, 1ull << 31)));
    g.dzr.init(g.nz % kZGroup ? g.nz % kZGroup : 1u);
    g.zgroup = static_cast<uint64_t>(g.nx) * g.ny >= kZGroupMinPlane ? 1u : 0u;
    for (int a = 0; a < 3; ++a) g.wall[a] = desc->wall[a];
    g.moving = 0;
    for (int f = 0; f < 6; ++f)
        for (int b = 0; b < 3; ++b) {
            g.wu[f][b] = desc->wall_velocity[f][b];
            if (desc->wall_velocity[f][b] != 0.0) g.moving |= 1 << f;
        }
    std::snprintf(c->err, sizeof(c->err), "no error");
    const size_t pb = partial_blocks(c);
    hipError_t e = hipMalloc(&c->partials, sizeof(double) * kPartialStride * (pb + (pb + kBlock - 1) / kBlock));
    if (e != hipSuccess) {
        rc = hip_fail(nullptr, e, "hipMalloc(partials)");
        delete c;
        return rc;
    }
    e = hipMalloc(&c->scal, sizeof(double) * 16);
    if (e != hipSuccess) {
        rc = hip_fail(nullptr, e, "hipMalloc(scalars)");
        (void)hipFree(c->partials);
        delete c;
        return rc;
    }
    c->links = nullptr;
    c->options = 0;
    {
        int dev = 0;
        c->num_cu = 0;
        e = hipGetDevice(&dev);
        if (e == hipSuccess) e = scratch_address(dev, &c->scratch);
        if (e != hipSuccess) {
            rc = hip_fail(nullptr, e, "device or static scratch address");
            (void)hipFree(c->partials);
            (void)hipFree(c->scal);
            delete c;
            return rc;
        }
        c->device = dev;
        if (hipDeviceGetAttribute(&c->num_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            c->num_cu = 0;
        if (c->num_cu <= 0) c->num_cu = 256;
        std::memset(c->t2_slots, 0, sizeof(c->t2_slots));
    }
    // the link table: for solid nodes, and for walls on lattices that take the fused kernel
    const bool walls = desc->wall[0] || desc->wall[1] || desc->wall[2];
    if (desc->solid || (walls && fused_kind(*desc))) {
        e = hipMalloc(&c->links, sizeof(uint32_t) * c->nodes);
        if (e == hipSuccess) {
            if (desc->lattice == CLBM_D3Q19)
                hipLaunchKernelGGL(k_links<19>, dim3(node_blocks(c)), dim3(kBlock), 0, c->stream, c->geom, desc->solid,
                                   c->links);
            else
                hipLaunchKernelGGL(k_links<27>, dim3(node_blocks(c)), dim3(kBlock), 0, c->stream, c->geom, desc->solid,
                                   c->links);
            e = hipGetLastError();
        }
        if (e != hipSuccess) {
            rc = hip_fail(nullptr, e, "link table");
            if (c->links) (void)hipFree(c->links);
            (void)hipFree(c->partials);
            (void)hipFree(c->scal);
            delete c;
            return rc;
        }
    }
    *out = c;
    return CLBM_OK;
}

int clbm_destroy(clbm_ctx *ctx)
{
    if (!ctx) return CLBM_OK;
    int rc = CLBM_OK;
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) rc = hip_fail(nullptr, e, "hipStreamSynchronize");
    (void)hipFree(ctx->partials);
    (void)hipFree(ctx->scal);
    if (ctx->links) (void)hipFree(ctx->links);
    delete ctx;
    return rc;
}

int clbm_set_stream(clbm_ctx *ctx, void *stream)
{
    if (!ctx) return fail(nullptr, CLBM_EINVAL, "ctx is NULL");
    ctx->stream = static_cast<hipStream_t>(stream);
    return CLBM_OK;
}

int clbm_set_rates(clbm_ctx *ctx, const double *s)
{
    if (!ctx || !s) return fail(ctx, CLBM_EINVAL, "ctx or rates is NULL");
    int rc = validate_rates(ctx, s);
    if (rc) return rc;
    std::memcpy(ctx->d.s, s, sizeof(double) * 10);
    return CLBM_OK;
}

int clbm_set_force(clbm_ctx *ctx, const double *uniform, const void *field, double scale)
{
    if (!ctx) return fail(nullptr, CLBM_EINVAL, "ctx is NULL");
    if (field && !aligned(field)) return fail(ctx, CLBM_EINVAL, "force field not 16-byte aligned");
    if (!std::isfinite(scale)) return fail(ctx, CLBM_EINVAL, "force scale not finite");
    double u[3] = {0.0, 0.0, 0.0};
    if (uniform)
        for (int a = 0; a < 3; ++a) {
            if (!std::isfinite(uniform[a])) return fail(ctx, CLBM_EINVAL, "uniform force not finite");
            u[a] = uniform[a];
        }
    std::memcpy(ctx->d.force_uniform, u, sizeof(u));
    ctx->d.force = field;
    ctx->d.force_scale = scale;
    return CLBM_OK;
}

int clbm_init(clbm_ctx *ctx, void *state, const double *rho0, const double *u0)
{
    if (!ctx) return fail(nullptr, CLBM_EINVAL, "ctx is NULL");
    if (!state || !aligned(state)) return fail(ctx, CLBM_EINVAL, "state NULL or not 16-byte aligned");
    if ((rho0 && !aligned(rho0)) || (u0 && !aligned(u0))) return fail(ctx, CLBM_EINVAL, "rho0/u0 not aligned");
    return dispatch(ctx, [&](auto v) {
        using Vt = decltype(v);
        using S = typename Vt::Store;
        if constexpr (Vt::q == 27) {
            if (ctx->d.collision == CLBM_MRT) {
                hipLaunchKernelGGL((k_init<S, Vt::check, Vt::solid, 27, true>), dim3(node_blocks(ctx)), dim3(kBlock),
                                   0, ctx->stream, static_cast<S *>(state), ctx->geom, ctx->links, rho0, u0);
                return check_launch(ctx, "init kernel launch");
            }
        }
        hipLaunchKernelGGL((k_init<S, Vt::check, Vt::solid, Vt::q, false>), dim3(node_blocks(ctx)), dim3(kBlock), 0,
                           ctx->stream, static_cast<S *>(state), ctx->geom, ctx->links, rho0, u0);
        return check_launch(ctx, "init kernel launch");
    });
}

int clbm_step(clbm_ctx *ctx, const void *src, void *dst)
{
    if (!ctx) return fail(nullptr, CLBM_EINVAL, "ctx is NULL");
    if (!src || !dst || !aligned(src) || !aligned(dst)) return fail(ctx, CLBM_EINVAL, "state NULL or misaligned");
    if (src == dst) return fail(ctx, CLBM_EINVAL, "src and dst must be distinct");
    return launch_step(ctx, src, dst);
}

int clbm_run(clbm_ctx *ctx, void *a, void *b, int32_t nsteps, void **result)
{
    if (!ctx) return fail(nullptr, CLBM_EINVAL, "ctx is NULL");
    if (!a || !b || !aligned(a) || !aligned(b) || a == b) return fail(ctx, CLBM_EINVAL, "bad state buffers");
    if (nsteps < 0) return fail(ctx, CLBM_EINVAL, "nsteps < 0");
    void *cur = a, *nxt = b;
    int32_t k = 0;
    if (fused_pairs(ctx))
        for (; k + 2 <= nsteps; k += 2) {
            const int rc = launch_step2(ctx, cur, nxt);
            if (rc) return rc;
            void *t = cur;
            cur = nxt;
            nxt = t;
        }
    for (; k < nsteps; ++k) {
        const int rc = launch_step(ctx, cur, nxt);
        if (rc) return rc;
        void *t = cur;
        cur = nxt;
        nxt = t;
    }
    if (result) *result = cur;
    return CLBM_OK;
}

int clbm_trajectory(clbm_ctx *ctx, const void *src, void *const *states, int32_t nsteps)
{
    if (!ctx) return fail(nullptr, CLBM_EINVAL, "ctx is NULL");
    if (nsteps < 0) return fail(ctx, CLBM_EINVAL, "nsteps < 0");
    if (!src || !aligned(src)) return fail(ctx, CLBM_EINVAL, "src NULL or misaligned");
    if (nsteps == 0) return CLBM_OK;
    if (!states) return fail(ctx, CLBM_EINVAL, "states is NULL");
    // every buffer distinct: a launch reads one of them while writing another
    for (int32_t k = 0; k < nsteps; ++k)
        if (!states[k] || !aligned(states[k])) return fail(ctx, CLBM_EINVAL, "a state buffer is NULL or misaligned");
    std::vector<uintptr_t> seen;
    try {
        seen.reserve(static_cast<size_t>(nsteps) + 1);
    } catch (...) {  // no exception crosses the C ABI
        return fail(ctx, CLBM_EINVAL, "out of host memory");
    }
    seen.push_back(reinterpret_cast<uintptr_t>(src));
    for (int32_t k = 0; k < nsteps; ++k) seen.push_back(reinterpret_cast<uintptr_t>(states[k]));
    std::sort(seen.begin(), seen.end());
    if (std::adjacent_find(seen.begin(), seen.end()) != seen.end())
        return fail(ctx, CLBM_EINVAL, "src and the state buffers must be distinct");
    // single steps: each state has to be written anyway, and a fused pair that also stores the state
    // between its steps moved its 1.5x bytes at the fused kernel's lower bandwidth, slower than two
    // single steps
    const void *cur = src;
    for (int32_t k = 0; k < nsteps; ++k) {
        const int rc = launch_step(ctx, cur, states[k]);
        if (rc) return rc;
        cur = states[k];
    }
    return CLBM_OK;
}

int clbm_set_options(clbm_ctx *ctx, uint32_t options)
{
    if (!ctx) return fail(nullptr, CLBM_EINVAL, "ctx is NULL");
    if (options & ~static_cast<uint32_t>(CLBM_OPT_SINGLE_STEP | CLBM_OPT_FUSED_PAIRS))
        return fail(ctx, CLBM_EINVAL, "unknown option bits");
    if ((options & CLBM_OPT_SINGLE_STEP) && (options & CLBM_OPT_FUSED_PAIRS))
        return fail(ctx, CLBM_EINVAL, "CLBM_OPT_SINGLE_STEP and CLBM_OPT_FUSED_PAIRS together");
    ctx->options = options;
    return CLBM_OK;
}

int clbm_fused_pairs(const clbm_ctx *ctx)
{
    if (!ctx) return fail(nullptr, CLBM_EINVAL, "ctx is NULL");
    return fused_pairs(ctx) ? 1 : 0;
}

int clbm_copy(clbm_ctx *ctx, const void *src, void *dst)
{
    if (!ctx) return fail(nullptr, CLBM_EINVAL, "ctx is NULL");
    if (!src || !dst || !aligned(src) || !aligned(dst) || src == dst)
        return fail(ctx, CLBM_EINVAL, "bad copy buffers");
    const size_t bytes = static_cast<size_t>(ctx->geom.P) * lattice_q(ctx->d) * store_size(ctx->d.storage);
    const size_t n16 = bytes / 16, tail = bytes % 16;
    if (n16) {
        size_t blocks = (n16 + kBlock - 1) / kBlock;
        if (blocks > 65536) blocks = 65536;
        hipLaunchKernelGGL(k_copy16, dim3(static_cast<unsigned>(blocks)), dim3(kBlock), 0, ctx->stream,
                           static_cast<const uint4 *>(src), static_cast<uint4 *>(dst), n16);
        int rc = check_launch(ctx, "copy kernel launch");
        if (rc) return rc;
    }
    if (tail) {
        hipLaunchKernelGGL(k_copy_tail, dim3(1), dim3(64), 0, ctx->stream,
                           static_cast<const uint8_t *>(src) + 16 * n16, static_cast<uint8_t *>(dst) + 16 * n16, tail);
        return check_launch(ctx, "copy tail launch");
    }
    return CLBM_OK;
}

int clbm_moments(clbm_ctx *ctx, const void *state, double *rho, double *u, double *totals, int64_t *n_bad)
{
    if (!ctx) return fail(nullptr, CLBM_EINVAL, "ctx is NULL");
    if (!state || !aligned(state)) return fail(ctx, CLBM_EINVAL, "state NULL or misaligned");
    if ((rho && !aligned(rho)) || (u && !aligned(u))) return fail(ctx, CLBM_EINVAL, "rho/u not aligned");
    const unsigned nb = stride_blocks(ctx);
    int rc = dispatch(ctx, [&](auto v) {
        using Vt = decltype(v);
        using S = typename Vt::Store;
        using R = typename Vt::R;
        hipLaunchKernelGGL((k_moments<S, Vt::check, Vt::solid, Vt::field, Vt::q>), dim3(nb), dim3(kBlock), 0, ctx->stream,
                           static_cast<const S *>(state), ctx->geom, ctx->links, static_cast<const R *>(ctx->d.force),
                           make_forcing<R>(ctx->d), rho, u, ctx->partials);
        return check_launch(ctx, "moments kernel launch");
    });
    if (rc) return rc;
    if (!totals && !n_bad) return CLBM_OK;
    // partials use a stride of kMomComp per block: reduce with that stride
    hipLaunchKernelGGL(k_reduce, dim3(kMomComp), dim3(kBlock), 0, ctx->stream, ctx->partials, static_cast<int>(nb),
                       kMomComp, ctx->scal, 0);
    rc = check_launch(ctx, "reduce kernel launch");
    if (rc) return rc;
    double h[kMomComp];
    hipError_t e = hipMemcpyAsync(h, ctx->scal, sizeof(h), hipMemcpyDeviceToHost, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipMemcpyAsync(totals)");
    e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamSynchronize");
    if (totals)
        for (int k = 0; k < 4; ++k) totals[k] = h[k];
    const int64_t bad = static_cast<int64_t>(h[4]);
    if (n_bad) *n_bad = bad;
    if (bad > 0) return fail(ctx, CLBM_ENONFINITE, "non-finite or non-positive density/velocity found");
    return CLBM_OK;
}

int clbm_get_populations(clbm_ctx *ctx, const void *state, double *f)
{
    if (!ctx) return fail(nullptr, CLBM_EINVAL, "ctx is NULL");
    if (!state || !f || !aligned(state) || !aligned(f)) return fail(ctx, CLBM_EINVAL, "bad buffers");
    return dispatch(ctx, [&](auto v) {
        using Vt = decltype(v);
        using S = typename Vt::Store;
        hipLaunchKernelGGL((k_get_populations<S, Vt::check, Vt::solid, Vt::q>), dim3(node_blocks(ctx)), dim3(kBlock), 0,
                           ctx->stream, static_cast<const S *>(state), ctx->geom, ctx->links, f);
        return check_launch(ctx, "get_populations kernel launch");
    });
}

int clbm_sample_populations(clbm_ctx *ctx, const void *state, const int32_t *nodes, int32_t count, double *out)
{
    if (!ctx) return fail(nullptr, CLBM_EINVAL, "ctx is NULL");
    if (!state || !aligned(state) || count < 0) return fail(ctx, CLBM_EINVAL, "bad state or count");
    if (count == 0) return CLBM_OK;
    if (!nodes || !out || (reinterpret_cast<uintptr_t>(nodes) & 3u) || (reinterpret_cast<uintptr_t>(out) & 7u))
        return fail(ctx, CLBM_EINVAL, "bad nodes/out buffers");
    return dispatch(ctx, [&](auto v) {
        using Vt = decltype(v);
        using S = typename Vt::Store;
        const unsigned blocks = static_cast<unsigned>((count + kBlock - 1) / kBlock);
        hipLaunchKernelGGL((k_sample_populations<S, Vt::check, Vt::solid, Vt::q>), dim3(blocks), dim3(kBlock), 0,
                           ctx->stream, static_cast<const S *>(state), ctx->geom, ctx->links, nodes,
                           static_cast<uint32_t>(count), out);
        return check_launch(ctx, "sample_populations kernel launch");
    });
}

int clbm_set_populations(clbm_ctx *ctx, const double *f, void *state)
{
    if (!ctx) return fail(nullptr, CLBM_EINVAL, "ctx is NULL");
    if (!state || !f || !aligned(state) || !aligned(f)) return fail(ctx, CLBM_EINVAL, "bad buffers");
    return dispatch(ctx, [&](auto v) {
        using Vt = decltype(v);
        using S = typename Vt::Store;
        hipLaunchKernelGGL((k_set_populations<S, Vt::check, Vt::solid, Vt::q>), dim3(node_blocks(ctx)), dim3(kBlock), 0,
                           ctx->stream, f, ctx->geom, ctx->links, static_cast<S *>(state));
        return check_launch(ctx, "set_populations kernel launch");
    });
}

}  // extern "C"

namespace {

int check_adjoint_args(clbm_ctx *ctx, const void *state_t, const void *lam_next, const void *lam_out,
                       const void *dJdF, const double *dJds)
{
    if (!state_t || !lam_next || !lam_out || !aligned(state_t) || !aligned(lam_next) || !aligned(lam_out))
        return fail(ctx, CLBM_EINVAL, "bad adjoint buffers");
    if (lam_next == lam_out) return fail(ctx, CLBM_EINVAL, "lam_next and lam_out must be distinct");
    if ((dJdF && !aligned(dJdF)) || (dJds && !aligned(dJds))) return fail(ctx, CLBM_EINVAL, "dJdF/dJds misaligned");
    return CLBM_OK;
}

// The adjoint step with its dJ/ds partial sums in `partials` (one row per block) and, when there are more
// rows than one reduction pass takes, their folded rows in `folded`.
int adjoint_step_with(clbm_ctx *ctx, const void *state_t, const void *lam_next, void *lam_out, void *dJdF,
                      double *dJds, double *partials, double *folded)
{
    const unsigned nb = node_blocks(ctx);
    int rc = dispatch_d3q27(ctx, [&](auto v) {
        using Vt = decltype(v);
        using S = typename Vt::Store;
        using R = typename Vt::R;
        hipLaunchKernelGGL((k_adjoint<S, Vt::check, Vt::solid, Vt::field>), dim3(nb), dim3(kBlock), 0, ctx->stream,
                           static_cast<const S *>(state_t), ctx->geom, ctx->links,
                           static_cast<const R *>(ctx->d.force), make_forcing<R>(ctx->d), make_rates<R>(ctx->d.s),
                           static_cast<const R *>(lam_next), static_cast<R *>(lam_out), static_cast<R *>(dJdF),
                           partials);
        return check_launch(ctx, "adjoint kernel launch");
    });
    if (rc || !dJds) return rc;
    const double *rows = partials;
    unsigned nrows = nb;
    if (nb > static_cast<unsigned>(kMaxBlocks)) {  // fold the long table first (fixed order)
        nrows = (nb + kBlock - 1) / kBlock;
        hipLaunchKernelGGL(k_fold<kAdjRates>, dim3(nrows), dim3(kBlock), 0, ctx->stream, partials,
                           static_cast<int>(nb), folded);
        rc = check_launch(ctx, "fold kernel launch");
        if (rc) return rc;
        rows = folded;
    }
    hipLaunchKernelGGL(k_reduce, dim3(kAdjRates), dim3(kBlock), 0, ctx->stream, rows, static_cast<int>(nrows),
                       kAdjRates, dJds + 2, 1);
    return check_launch(ctx, "reduce kernel launch");
}

}  // namespace

extern "C" {

int clbm_adjoint_step(clbm_ctx *ctx, const void *state_t, const void *lam_next, void *lam_out, void *dJdF,
                      double *dJds)
{
    if (!ctx) return fail(nullptr, CLBM_EINVAL, "ctx is NULL");
    const int rc = check_adjoint_args(ctx, state_t, lam_next, lam_out, dJdF, dJds);
    if (rc) return rc;
    return adjoint_step_with(ctx, state_t, lam_next, lam_out, dJdF, dJds, ctx->partials,
                             ctx->partials + partial_blocks(ctx) * kPartialStride);
}

int clbm_adjoint_step_noalloc(clbm_ctx *ctx, const void *state_t, const void *lam_next, void *lam_out, void *dJdF,
                              double *dJds)
{
    if (!ctx) return fail(nullptr, CLBM_EINVAL, "ctx is NULL");
    if (ctx->nodes > kNoallocMaxNodes)
        return fail(ctx, CLBM_EINVAL,
                    "lattice larger than the 2^25 nodes the static scratch of clbm_adjoint_step_noalloc holds%s",
                    " (use clbm_adjoint_step)");
    const int rc = check_adjoint_args(ctx, state_t, lam_next, lam_out, dJdF, dJds);
    if (rc) return rc;
    // scratch: a device address from hipGetSymbolAddress (set up by clbm_create on this device)
    return adjoint_step_with(ctx, state_t, lam_next, lam_out, dJdF, dJds, ctx->scratch,
                             ctx->scratch + kNoallocRows * kAdjRates);
}

int64_t clbm_adjoint_noalloc_max_nodes(void) { return static_cast<int64_t>(kNoallocMaxNodes); }

int clbm_loss_seed(clbm_ctx *ctx, const void *state, const void *u_target, void *lam_out, void *dJdF, double *J)
{
    if (!ctx) return fail(nullptr, CLBM_EINVAL, "ctx is NULL");
    if (!state || !u_target || !lam_out || !aligned(state) || !aligned(u_target) || !aligned(lam_out))
        return fail(ctx, CLBM_EINVAL, "bad loss buffers");
    if ((dJdF && !aligned(dJdF)) || (J && (reinterpret_cast<uintptr_t>(J) & 7u)))
        return fail(ctx, CLBM_EINVAL, "dJdF/J misaligned");
    const unsigned nb = stride_blocks(ctx);
    int rc = dispatch_d3q27(ctx, [&](auto v) {
        using Vt = decltype(v);
        using S = typename Vt::Store;
        using R = typename Vt::R;
        hipLaunchKernelGGL((k_loss<S, Vt::check, Vt::solid, Vt::field>), dim3(nb), dim3(kBlock), 0, ctx->stream,
                           static_cast<const S *>(state), ctx->geom, ctx->links, static_cast<const R *>(ctx->d.force),
                           make_forcing<R>(ctx->d), static_cast<const R *>(u_target), static_cast<R *>(lam_out),
                           static_cast<R *>(dJdF), ctx->partials);
        return check_launch(ctx, "loss kernel launch");
    });
    if (rc || !J) return rc;
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kBlock), 0, ctx->stream, ctx->partials, static_cast<int>(nb), 1, J, 1);
    return check_launch(ctx, "reduce kernel launch");
}

}  // extern "C"

// Host-side logic of the library that needs no GPU: descriptor and rate checks,
// the plane stride helper, status strings and the z-chunking of the fused
// two-step launch.  Plain C++ with no HIP types, included by clbm.hip; the CPU
// test tests/test_host_sanitizers.py also builds it with g++ under AddressSanitizer
// and UndefinedBehaviorSanitizer.
#pragma once

#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstdio>

#include "../../include/clbm.h"

namespace clbm_host {

constexpr size_t kErrLen = 512;

inline int fail(char *err, int code, const char *fmt, const char *arg = "")
{
    std::snprintf(err, kErrLen, fmt, arg);
    return code;
}

inline bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

inline size_t store_size(int storage) { return storage == CLBM_F64 ? 8 : (storage == CLBM_F32 ? 4 : 2); }

// nx * ny * nz for dims >= 1, or -1 when it reaches 2^31 (checked before each product, so that
// no product of three int32 values can overflow)
inline long long node_count(int32_t nx, int32_t ny, int32_t nz)
{
    const long long nxy = static_cast<long long>(nx) * ny;  // < 2^62
    if (nxy >= (1ll << 31)) return -1;
    const long long n = nxy * nz;  // < 2^62
    return n >= (1ll << 31) ? -1 : n;
}

// Each rate of Eq. (13) must lie in (0, 2) (NaN fails too).
inline int validate_rates(char *err, const double *s)
{
    static const char *const names[10] = {"s0", "s1", "s2", "s2b", "s3", "s3b", "s4", "s4b", "s5", "s6"};
    for (int k = 0; k < 10; ++k)
        if (!(s[k] > 0.0 && s[k] < 2.0)) return fail(err, CLBM_ERATE, "relaxation rate %s outside (0, 2)", names[k]);
    return CLBM_OK;
}

inline int validate_desc(const clbm_desc *d, char *err)
{
    if (!d) return fail(err, CLBM_EINVAL, "desc is NULL");
    if (d->nx < 1 || d->ny < 1 || d->nz < 1) return fail(err, CLBM_EINVAL, "lattice dims must be >= 1");
    const long long n = node_count(d->nx, d->ny, d->nz);
    if (n < 0) return fail(err, CLBM_EINVAL, "nx*ny*nz must be below 2^31");
    for (int a = 0; a < 3; ++a)
        if (d->wall[a] != 0 && d->wall[a] != 1) return fail(err, CLBM_EINVAL, "wall flags must be 0 or 1");
    if (d->storage < CLBM_F64 || d->storage > CLBM_BF16) return fail(err, CLBM_EDTYPE, "unknown storage type");
    // kernels address a plane (state, adjoint, force field: elements of at most 8 bytes for FP64
    // storage, 4 otherwise) with 32-bit byte offsets
    const long long widest = d->storage == CLBM_F64 ? 8 : 4;
    if (n * widest > (1ll << 32))
        return fail(err, CLBM_EINVAL, "lattice too large: nx*ny*nz times the element size must not exceed 4 GiB");
    if (d->lattice != CLBM_D3Q27 && d->lattice != CLBM_D3Q19) return fail(err, CLBM_EINVAL, "unknown lattice");
    if (d->collision != CLBM_CASCADED && d->collision != CLBM_MRT)
        return fail(err, CLBM_EINVAL, "unknown collision model");
    if (d->collision == CLBM_MRT && d->lattice != CLBM_D3Q27)
        return fail(err, CLBM_EINVAL, "the MRT collision needs the D3Q27 lattice");
    if (d->reserved != 0) return fail(err, CLBM_EINVAL, "reserved field must be 0");
    if (d->plane_stride != 0) {
        const size_t es = store_size(d->storage);
        if (d->plane_stride < n || d->plane_stride > 0xffffffffll)
            return fail(err, CLBM_EINVAL, "plane_stride must lie in [nx*ny*nz, 2^32)");
        if ((static_cast<size_t>(d->plane_stride) * es) % 16 != 0)
            return fail(err, CLBM_EINVAL, "plane_stride * element size must be a multiple of 16 bytes");
    }
    for (int f = 0; f < 6; ++f)
        for (int b = 0; b < 3; ++b) {
            const double w = d->wall_velocity[f][b];
            if (!std::isfinite(w)) return fail(err, CLBM_EINVAL, "wall velocity not finite");
            if (w != 0.0 && !d->wall[f / 2]) return fail(err, CLBM_EINVAL, "a face of a periodic axis cannot move");
        }
    int rc = validate_rates(err, d->s);
    if (rc) return rc;
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(d->force_uniform[a])) return fail(err, CLBM_EINVAL, "force_uniform not finite");
    if (!std::isfinite(d->force_scale)) return fail(err, CLBM_EINVAL, "force_scale not finite");
    if (d->force && !aligned16(d->force)) return fail(err, CLBM_EINVAL, "force field not 16-byte aligned");
    return CLBM_OK;
}

// Default plane stride: N rounded up to 256 bytes plus 4 KiB, so that the 27 planes of a state do not
// start at power-of-two distances; -1 for invalid arguments.
inline int64_t default_plane_stride(int32_t nx, int32_t ny, int32_t nz, int32_t storage)
{
    if (nx < 1 || ny < 1 || nz < 1 || storage < CLBM_F64 || storage > CLBM_BF16) return -1;
    const long long n = node_count(nx, ny, nz);
    if (n < 0) return -1;
    const long long es = static_cast<long long>(store_size(storage));
    const long long align = 256 / es, pad = 4096 / es;
    return (n + align - 1) / align * align + pad;
}

inline const char *status_string(int status)
{
    switch (status) {
    case CLBM_OK: return "success";
    case CLBM_EINVAL: return "invalid argument";
    case CLBM_ERATE: return "relaxation rate outside (0, 2)";
    case CLBM_EDTYPE: return "unknown storage type";
    case CLBM_EHIP: return "HIP runtime error";
    case CLBM_ENONFINITE: return "non-finite or non-positive density/velocity found";
    default: return "unknown status";
    }
}

// A block of the fused kernel runs through a whole z chunk, so a launch whose last
// round of blocks fills only part of the GPU idles for the rest of that round.
// Choose the chunks per tile column (each of at least 8 planes) to minimise
// rounds x (planes per chunk + 2), the two extra planes being the halo planes a
// chunk recomputes; slots = blocks resident on the device at once (>= 1).
// Returns the number of chunks; ceil(nz / chunks) planes each cover nz.
inline uint32_t fused_chunks(uint32_t tiles, uint32_t nz, uint32_t slots)
{
    const uint32_t max_chunks = nz / 8 > 1 ? nz / 8 : 1;
    uint32_t best = 1;
    unsigned long long best_cost = ~0ull;
    for (uint32_t nc = 1; nc <= max_chunks; ++nc) {
        const uint32_t zchunk = (nz + nc - 1) / nc;
        const uint32_t used = (nz + zchunk - 1) / zchunk;
        const unsigned long long rounds = (static_cast<unsigned long long>(tiles) * used + slots - 1) / slots;
        const unsigned long long cost = rounds * (zchunk + 2);
        if (cost < best_cost) {
            best_cost = cost;
            best = used;
        }
    }
    return best;
}

}  // namespace clbm_host

// LDS staging for the nearest-neighbour stencils (Wilson, staggered).
//
// A work-group owns a tile of S consecutive sites (linear site order) and all their
// right-hand sides.  For every hop direction the S neighbour site blocks (each block is a
// contiguous [colour][spin][rhs] record of `block` bytes) are copied into LDS by the whole
// work-group with unit-stride loads of `Unit` (16 or 8 bytes), so each wavefront load
// instruction reads one contiguous stretch of memory.  Threads then read the components of
// their (site, rhs group) from LDS.  The output block of the tile is staged the same way so
// the stores are contiguous too.  Row stride in LDS is padded by one unit to spread banks.
#pragma once

#include "common.h"
#include "kernels.h"

namespace dirac {

// Direction slots of the neighbour table: 0 = the site itself, 1 + 2 mu = n + mu, 2 + 2 mu = n - mu.
constexpr int kHopSlots = 9;

struct TileGeom {
    int S;            // sites per tile
    int nrg;          // right-hand-side groups per site (threads per site)
    int units;        // Unit-sized words per site block
    uint32_t magic;   // ceil(2^32 / units): q = umulhi(u, magic) == u / units for u < S * units
    uint32_t magic_nrg;  // same for nrg
};

// u / d for u < 2^32 / d using the precomputed reciprocal ceil(2^32 / d); d = 1 is encoded as
// magic = 0 (its reciprocal does not fit in 32 bits).
__device__ __forceinline__ uint32_t fast_div(uint32_t u, uint32_t magic) { return magic ? __umulhi(u, magic) : u; }

inline uint32_t div_magic(uint32_t d) { return d <= 1 ? 0u : static_cast<uint32_t>((0x100000000ull + d - 1) / d); }

// Neighbour table of a tile: nb[slot * S + j] for the S sites starting at s0 (sites past the
// end of the lattice map to site 0 and are never stored).
__device__ __forceinline__ void tile_neighbours(int* nb, int64_t s0, int S, const Geom& g) {
    for (int j = threadIdx.x; j < S; j += blockDim.x) {
        int64_t s = s0 + j;
        if (s >= g.vol) s = 0;
        const Coord c = site_coord(s, g);
        nb[j] = static_cast<int>(s);
        const int ext[4] = {g.nx, g.ny, g.nz, g.nt};
        const int co[4] = {c.x, c.y, c.z, c.t};
        const int64_t stride[4] = {1, g.nx, static_cast<int64_t>(g.nx) * g.ny,
                                   static_cast<int64_t>(g.nx) * g.ny * g.nz};
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            const int64_t f = s + (co[mu] == ext[mu] - 1 ? (1 - ext[mu]) * stride[mu] : stride[mu]);
            const int64_t b = s - (co[mu] == 0 ? (1 - ext[mu]) * stride[mu] : stride[mu]);
            nb[(1 + 2 * mu) * S + j] = static_cast<int>(f);
            nb[(2 + 2 * mu) * S + j] = static_cast<int>(b);
        }
    }
}

// Copy the blocks of sites nb[0..S) (each `units` Units long) from global `src` into LDS `dst`
// with row stride units + 1.
template <typename Unit>
__device__ __forceinline__ void tile_gather(Unit* __restrict__ dst, const Unit* __restrict__ src, const int* nb,
                                            const TileGeom& tg) {
    const uint32_t total = static_cast<uint32_t>(tg.S) * tg.units;
    for (uint32_t u = threadIdx.x; u < total; u += blockDim.x) {
        const uint32_t j = fast_div(u, tg.magic);
        const uint32_t k = u - j * tg.units;
        dst[j * (tg.units + 1) + k] = src[static_cast<int64_t>(nb[j]) * tg.units + k];
    }
}

// Copy a contiguous range of `count` Units from global to LDS.
template <typename Unit>
__device__ __forceinline__ void copy_in(Unit* __restrict__ dst, const Unit* __restrict__ src, uint32_t count) {
    for (uint32_t u = threadIdx.x; u < count; u += blockDim.x) dst[u] = src[u];
}

// Store the staged tile (row stride units + 1) to the contiguous output range of the tile.
template <typename Unit>
__device__ __forceinline__ void tile_scatter_out(Unit* __restrict__ dst, const Unit* __restrict__ lds, int nsites,
                                                 const TileGeom& tg) {
    const uint32_t total = static_cast<uint32_t>(nsites) * tg.units;
    for (uint32_t u = threadIdx.x; u < total; u += blockDim.x) {
        const uint32_t j = fast_div(u, tg.magic);
        const uint32_t k = u - j * tg.units;
        dst[u] = lds[j * (tg.units + 1) + k];
    }
}

// LDS bytes of a tile of S sites: neighbour table, forward links (fwd_bytes per site),
// backward links of one direction (bwd_bytes per site) and the padded spinor tile.
inline size_t lds_bytes(int S, size_t fwd_bytes, size_t bwd_bytes, int units, size_t unit_bytes) {
    auto up = [](size_t b) { return (b + 15) / 16 * 16; };
    return up(static_cast<size_t>(kHopSlots) * S * sizeof(int)) + up(S * fwd_bytes) + up(S * bwd_bytes) +
           static_cast<size_t>(S) * (units + 1) * unit_bytes;
}

constexpr size_t kTileLdsBudget = 64 * 1024;
constexpr int kTileMaxThreads = 512;

// Sites per tile: a multiple of 64/gcd(64, nrg) (whole wavefronts) up to 256 threads, within
// the LDS budget; smaller tiles if the RHS block is large.  0 if not even one site fits.
template <typename F>
int choose_tile_sites(int nrg, F lds_of) {
    int g = 64;
    for (int a = nrg, b = 64; b;) {
        const int t = a % b;
        a = b;
        b = t;
        g = a;
    }
    int base = 64 / g;
    int S = 0;
    for (int s = base; s * nrg <= 256 && lds_of(s) <= kTileLdsBudget; s *= 2) S = s;
    if (S == 0) {
        for (int s = base; s >= 1; --s)
            if (s * nrg <= kTileMaxThreads && lds_of(s) <= kTileLdsBudget) {
                S = s;
                break;
            }
    }
    return S;
}

// The LDS-staged tiles are used when variant 2 is selected (see choose_variant).
inline bool use_lds_variant(const StencilArgs& a, bool = true) { return a.variant == 2; }

inline bool tile_aligned(const StencilArgs& a) {
    auto al = [](const void* p) { return reinterpret_cast<uintptr_t>(p) % 16 == 0; };
    return al(a.gauge) && al(a.in) && al(a.out);
}

}  // namespace dirac

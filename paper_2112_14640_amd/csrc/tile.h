// Row tiles of the stencil kernels (Wilson, staggered, Brillouin): geometry, tile order and the raw
// buffer loads that copy whole x-rows of the lattice into LDS.
#pragma once

#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace dirac {

// u / d for u < 2^32 / d using the precomputed reciprocal ceil(2^32 / d); d = 1 is encoded as
// magic = 0 (its reciprocal does not fit in 32 bits).
__device__ __forceinline__ uint32_t fast_div(uint32_t u, uint32_t magic) { return magic ? __umulhi(u, magic) : u; }

inline uint32_t div_magic(uint32_t d) { return d <= 1 ? 0u : static_cast<uint32_t>((0x100000000ull + d - 1) / d); }

// ---------------------------------------------------------------------------
// Row tiles.  Rows are the x-lines of the lattice, numbered rho = site / nx = y + ny (z + nz t).
// A work-group owns one row (S = nx sites) and every right-hand side of it.  Its own row also
// holds the +-x neighbours (periodic within the row); each of the other six hop directions needs
// one whole row, a contiguous stretch of memory, so every copy into LDS is a contiguous
// 16-byte-per-lane load.
// ---------------------------------------------------------------------------
struct RowTile {
    int R;                 // rows per tile (1)
    int S;                 // sites per tile, R * nx
    int nrg;               // RHS groups per site (threads per site)
    int units;             // 16-byte units per site block
    int row_units;         // nx * units
    int threads;           // S * nrg active threads
    int64_t ntiles;        // rows / R (times nseg)
    int nseg;              // x-segments per row (Brillouin; 1 for the others)
    uint32_t magic_nrg, magic_nx, magic_units, magic_row_units;
    // Tile order.  The t range is cut into slabs of ts slices, one slab per XCD when nt allows
    // (the launch gives each XCD a contiguous eighth of the tiles), so only the +-t copies at a
    // slab face come from another XCD's share.  Inside a slab: (y, z) blocks of by x bz rows,
    // then t, then the rows of the block, so the rows a tile shares with its +-y, +-z and +-t
    // neighbours are fetched close together in time.
    int by, bz, nby, ts;
    // ceil(2^32 / d) for d = by * bz, by, ts, nby (0 when d = 1), exact over the ranges of
    // tile_row (row_order checks that); a slab division is done only when there are several slabs
    uint32_t magic_bsz, magic_by, magic_ts, magic_nby;
};

// Lattice coordinates of a row (x = 0).
struct RowPos {
    int y, z, t;
};

__device__ __forceinline__ uint32_t row_index(const RowPos& p, const Geom& g) {
    return static_cast<uint32_t>(p.y + g.ny * (p.z + g.nz * p.t));
}

// First site of the row one step from row p: dir 0..5 = +y, -y, +z, -z, +t, -t (periodic).
__device__ __forceinline__ int64_t row_neighbour_start(const RowPos& p, int dir, const Geom& g) {
    int y = p.y, z = p.z, t = p.t;
    switch (dir) {
        case 0: y = y + 1 == g.ny ? 0 : y + 1; break;
        case 1: y = y == 0 ? g.ny - 1 : y - 1; break;
        case 2: z = z + 1 == g.nz ? 0 : z + 1; break;
        case 3: z = z == 0 ? g.nz - 1 : z - 1; break;
        case 4: t = t + 1 == g.nt ? 0 : t + 1; break;
        default: t = t == 0 ? g.nt - 1 : t - 1; break;
    }
    return ((static_cast<int64_t>(t) * g.nz + z) * g.ny + y) * g.nx;
}

// 16- and 8-byte units of the row copies (native vector types, so register arrays of them stay
// in registers).
using u32x4 = unsigned int __attribute__((ext_vector_type(4)));
using u32x2 = unsigned int __attribute__((ext_vector_type(2)));

// Raw buffer resource over `bytes` bytes from `base` (gfx9 descriptor: 32-bit data format, no
// stride).  Row copies load through it with a per-lane offset fixed for the kernel and a
// work-group-uniform offset, so their address arithmetic stays on the scalar unit; a read at or
// past `bytes` returns zero instead of touching memory.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_buffer(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, static_cast<int>(bytes), 0x00020000);
}

template <typename Unit>
__device__ __forceinline__ Unit buffer_load_unit(__amdgpu_buffer_rsrc_t r, uint32_t lane_off, uint32_t uni_off) {
    if constexpr (sizeof(Unit) == 16)
        return __builtin_bit_cast(Unit, __builtin_amdgcn_raw_buffer_load_b128(r, lane_off, uni_off, 0));
    else
        return __builtin_bit_cast(Unit, __builtin_amdgcn_raw_buffer_load_b64(r, lane_off, uni_off, 0));
}

// 16-byte units each thread moves per row copy of a four-spin field: its share of the row.
template <int NC, int RB, class P>
struct RowUnits {
    static constexpr int PER = NC * 4 * RB * static_cast<int>(sizeof(typename P::S)) / 16;
};

// Bytes of LDS for one staged row tile (site stride padded by one 16-byte unit).
// Padding (in row units of udw dwords) after each site of a row copy in LDS.  The threads of a wave
// read one element of consecutive RHS at a time, site after site; with the site stride congruent, modulo
// the 64 LDS banks, to the span (dwords) of one site's RHS run, the runs of consecutive sites fall on
// consecutive banks and a read is free of bank conflicts.  One unit when the span is not a whole number
// of units or already covers the 64 banks (a wider pad measured slower there).
__host__ __device__ inline uint32_t row_pad(uint32_t units, uint32_t span, uint32_t udw = 4) {
    if (span % udw != 0 || span > 64u) return 1u;
    return ((span % 64u) + 64u - (udw * units) % 64u) % 64u / udw;
}
inline size_t row_tile_lds(int S, int units, uint32_t pad) { return static_cast<size_t>(S) * (units + pad) * 16; }

// Row processed by tile number T (after the XCD remap) in the order of RowTile.  The divisors
// are uniform over the work-group; the magic multiplies keep them on the scalar unit.
__device__ __forceinline__ RowPos tile_row_pos(uint32_t T, const RowTile& rt, const Geom& g) {
    uint32_t slab = 0, T2 = T;
    if (rt.ts != g.nt) {
        const uint32_t slab_rows = static_cast<uint32_t>(g.ny * g.nz) * static_cast<uint32_t>(rt.ts);
        slab = T / slab_rows;
        T2 = T - slab * slab_rows;
    }
    const uint32_t bsz = static_cast<uint32_t>(rt.by * rt.bz);
    const uint32_t q = fast_div(T2, rt.magic_bsz);
    const uint32_t rin = T2 - q * bsz;
    const uint32_t b = fast_div(q, rt.magic_ts);
    const uint32_t t = slab * rt.ts + (q - b * static_cast<uint32_t>(rt.ts));
    const uint32_t bzi = fast_div(b, rt.magic_nby);
    const uint32_t byi = b - bzi * static_cast<uint32_t>(rt.nby);
    const uint32_t zin = fast_div(rin, rt.magic_by);
    const uint32_t y = byi * rt.by + (rin - zin * rt.by);
    const uint32_t z = bzi * rt.bz + zin;
    return {static_cast<int>(y), static_cast<int>(z), static_cast<int>(t)};
}

__device__ __forceinline__ uint32_t tile_row(uint32_t T, const RowTile& rt, const Geom& g) {
    return row_index(tile_row_pos(T, rt, g), g);
}

// Block extent of the row order along one axis: `want` (a power of two) or the largest power of
// two below it that divides n.
inline int row_block_extent(int n, int want) {
    while (want > 1 && n % want != 0) want /= 2;
    return want;
}

inline bool row_order_magic(const Geom& g, RowTile& rt);

// Row order: 4 x 4 (y, z) blocks over the whole t range (smaller powers of two where the extents
// need them).  False if its divisions cannot be done exactly with 32-bit magic multiplies (the row
// kernels are then not used).
inline bool row_order(int, const Geom& g, RowTile& rt) {
    rt.by = row_block_extent(g.ny, 4);
    rt.bz = row_block_extent(g.nz, 4);
    rt.ts = g.nt;
    rt.nby = g.ny / rt.by;
    return row_order_magic(g, rt);
}

// ceil(2^32 / d) when umulhi(u, magic) == u / d for every u < umax (0 for d = 1); false if not.
inline bool exact_magic(uint32_t d, uint64_t umax, uint32_t& magic) {
    magic = div_magic(d);
    if (d <= 1) return true;
    const uint64_t e = static_cast<uint64_t>(magic) * d - 0x100000000ull;
    return umax * e < 0x100000000ull;
}

// Magic divisors of tile_row_pos for the order row_order chose; false if one is not exact.
inline bool row_order_magic(const Geom& g, RowTile& rt) {
    const uint64_t slab_rows = static_cast<uint64_t>(g.ny) * g.nz * rt.ts;
    const uint32_t bsz = static_cast<uint32_t>(rt.by * rt.bz);
    return exact_magic(bsz, slab_rows, rt.magic_bsz) && exact_magic(rt.by, bsz, rt.magic_by) &&
           exact_magic(rt.ts, slab_rows / bsz, rt.magic_ts) &&
           exact_magic(rt.nby, static_cast<uint64_t>(rt.nby) * (g.nz / rt.bz), rt.magic_nby);
}

// LDS a work-group may request on the current device (64 KiB unless the device reports more;
// above 64 KiB a kernel must opt in with hipFuncAttributeMaxDynamicSharedMemorySize).
inline size_t max_lds_per_block() {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v < 65536)
        return 65536;
    return static_cast<size_t>(v);
}

// Largest row tile taken: 96 KiB of LDS (two work-groups per 160 KiB CU).
constexpr size_t kRowLdsCap = 96 * 1024;

// Row tiles are used (variant 4) when one row of every RHS fits: 64..512 threads and at
// most kRowLdsCap bytes of LDS (and what the device allows).  Returns the rows per tile (1) or 0.
inline int choose_tile_rows(int, int64_t rows, int nx, int units, int nrg, uint32_t pad) {
    const int64_t threads = static_cast<int64_t>(nx) * nrg;
    const size_t lds = row_tile_lds(nx, units, pad);
    if (rows >= 1 && threads >= 64 && threads <= 512 && lds <= kRowLdsCap && lds <= max_lds_per_block()) return 1;
    return 0;
}

// Opt a row kernel in to more than 64 KiB of dynamic LDS (once per kernel); false if refused.
template <typename K>
bool allow_lds(K kernel, size_t lds) {
    if (lds <= 64 * 1024) return true;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                               static_cast<int>(kRowLdsCap)) == hipSuccess;
}

// ---------------------------------------------------------------------------
// Solver epilogue of the row kernels (see Epilogue in kernels.h).  acc[k][e] is the thread's output
// for right-hand side rhs0 + k and element e (element e of a site block at offset e * nv); elem0 is the
// index of the thread's first element in the vector.  Each tile writes nv per-RHS sums, reduced over
// its sites in a fixed order through `red` (LDS, at least sites * nv doubles, free when called).
// ---------------------------------------------------------------------------
template <typename R, typename S>
__device__ __forceinline__ cx<R> as_stored(cx<R> v) {
    S t;
    io<R, S>::st(&t, v);
    return io<R, S>::ld(&t);
}

template <int RB, int NE, typename R, typename S>
__device__ __forceinline__ void row_epilogue(const Epilogue& epi, const cx<R> (&acc)[RB][NE], bool active,
                                             int64_t elem0, int nv, int rhs0, uint32_t j, int sites, int64_t tile,
                                             double* red) {
    using RS = std::conditional_t<sizeof(R) == 8, double2, float2>;  // the residual's storage
    double sq[RB];
#pragma unroll
    for (int k = 0; k < RB; ++k) sq[k] = 0.0;
    if (active) {
        if (epi.mode == 2) {
            RS* r = static_cast<RS*>(epi.r) + elem0;
            const double2* al = reinterpret_cast<const double2*>(epi.alpha) + rhs0;
#pragma unroll
            for (int k = 0; k < RB; ++k) {
                const double2 a = al[k];
                const cx<double> ma{-a.x, -a.y};
#pragma unroll
                for (int e = 0; e < NE; ++e) {
                    const cx<R> q = as_stored<R, S>(acc[k][e]);
                    cx<double> rv = io<double, RS>::ld(r + e * nv + k);
                    cfma(rv, ma, cx<double>{static_cast<double>(q.re), static_cast<double>(q.im)});
                    io<double, RS>::st(r + e * nv + k, rv);
                    const cx<double> sv = io<double, RS>::ld(r + e * nv + k);
                    sq[k] += sv.re * sv.re + sv.im * sv.im;
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < RB; ++k)
#pragma unroll
                for (int e = 0; e < NE; ++e) {
                    const cx<R> v = as_stored<R, S>(acc[k][e]);
                    sq[k] += static_cast<double>(v.re) * v.re + static_cast<double>(v.im) * v.im;
                }
        }
    }
    __syncthreads();  // red may alias the row tile
    if (active)
#pragma unroll
        for (int k = 0; k < RB; ++k) red[j * nv + rhs0 + k] = sq[k];
    __syncthreads();
    if (threadIdx.x < static_cast<uint32_t>(nv)) {
        double t = 0.0;
        for (int jj = 0; jj < sites; ++jj) t += red[jj * nv + threadIdx.x];
        epi.partial[tile * nv + threadIdx.x] = t;
    }
}

inline bool tile_aligned(const StencilArgs& a) {
    auto al = [](const void* p) { return reinterpret_cast<uintptr_t>(p) % 16 == 0; };
    return al(a.gauge) && al(a.in) && al(a.out);
}

}  // namespace dirac

// Clover term of the Wilson and Brillouin operators (Sec. 4, Eq. def_clov), applied from a
// precomputed per-site field.
//
// In the chiral basis of App. A every sigma_{mu nu} is block diagonal in chirality (its tensor form
// is sigma_0 (x) sigma_k or sigma_3 (x) sigma_k, the first factor acting on the chirality), so
// C(n) = -(c_SW/2) sum_{mu<nu} sigma_{mu nu} (x) F_{mu nu}(n) is two hermitian 2N_c x 2N_c blocks,
// one for the spin pair (0, 1) and one for (2, 3):
//   block_h = -(c_SW/2) [[C_h, A_h - i B_h], [A_h + i B_h, -C_h]]
//   A_0 = F14 - F23, B_0 = F13 + F24, C_0 = F34 - F12;  A_1 = -F14 - F23, B_1 = F13 - F24,
//   C_1 = -F34 - F12  (F_{mu nu} for mu, nu = 1..4 = x, y, z, t).
// Storage (per site, reals of the apply's arithmetic type): block 0 then block 1, each N^2 reals
// with N = 2 N_c: the N diagonal entries, then the entries (i, j), i < j, row by row as (re, im).
// Component i of a block is local spin i / N_c (spin 2h + i / N_c of the vector) and colour i % N_c.
// The field is built once per gauge field by dirac_clover_field (c_SW folded in).
#pragma once

#include "common.h"

namespace dirac {

template <int NC>
constexpr int clover_reals() {
    return 2 * (2 * NC) * (2 * NC);
}

// acc[k][a][s] += (C psi)[a][s] for the RB right-hand sides of one thread.  psi points at the
// thread's first RHS of the site block [colour][spin][rhs] (stride nv between (colour, spin)
// rows); c at the site's packed clover record.
template <int NC, int RB, typename R, typename S>
__device__ __forceinline__ void clover_add(cx<R> (&acc)[RB][NC][4], const S* __restrict__ psi, int nv,
                                           const R* __restrict__ c) {
    constexpr int N = 2 * NC;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const R* b = c + h * N * N;
#pragma unroll
        for (int k = 0; k < RB; ++k) {
            cx<R> v[N], o[N];
#pragma unroll
            for (int i = 0; i < N; ++i) {
                v[i] = io<R, S>::ld(psi + ((i % NC) * 4 + 2 * h + i / NC) * nv + k);
                o[i] = cscale(b[i], v[i]);
            }
            int e = N;
#pragma unroll
            for (int i = 0; i < N; ++i)
#pragma unroll
                for (int j = i + 1; j < N; ++j) {
                    const cx<R> bij{b[e], b[e + 1]};
                    e += 2;
                    cfma(o[i], bij, v[j]);
                    cfma_conj(o[j], bij, v[i]);
                }
#pragma unroll
            for (int i = 0; i < N; ++i) acc[k][i % NC][2 * h + i / NC] = cadd(acc[k][i % NC][2 * h + i / NC], o[i]);
        }
    }
}

}  // namespace dirac

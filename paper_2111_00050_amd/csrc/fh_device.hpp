// fh_device.hpp -- gfx950 kernels, templated on the number of modes M.
//
// Lexicographic rank (Sec. III.B sectors; sizes as in App. A).
// Let D_m(R, Q) count occupation vectors of modes m..M-1 with sum R and
// momentum sum_{j>=m} j n_j == Q (mod M).  The lexicographic rank of n inside
// its sector (N, P) (n_0 most significant) telescopes into
//     rank(n) = D_0(N, P) - 1 - sum_{s=1}^{M-1} T_s(R_s, Q_s),
//     T_s(R, Q) = D_{s-1}(R - 1, Q - (s - 1))   (0 for R <= 0),
// where (R_s, Q_s) are the suffix sums of n from mode s on.  T_s(R_s, Q_s)
// counts the sector states that agree with n on modes < s-1 and hold more
// bosons in mode s-1.  A neighbour n' that differs from n only in modes
// a..d changes (R_s, Q_s) only for a < s <= d, so its rank costs d - a table
// reads from the row's own terms.  The table (one int per (s, R, Q), with Q
// stored twice so that Q + dQ needs no reduction and R biased by two) lives in
// LDS; every offset (dR, dQ) of a neighbour is a compile-time constant folded
// into the ds_read immediate.
//
// H psi (Eq. Ham, projected on each sector as in Sec. III.B), gather form:
//   (H x)(n) = [sum_j w_j n_j + sum_{pairs} Wd_p occ_p(n)] x(n)
//            + sum_{row pair {i,j}} c_ij(n) sum_{source pair {k,l} of the class}
//                  W_{ij,kl} c_kl(n) x(n - e_i - e_j + e_k + e_l),
//   c_ij = sqrt(n_i (n_j - d_ij)), c_kl = sqrt((n_k + 1)(n_l + 1 + d_kl)),
//   W_{ij,kl} = (Lambda/2) sum over the orderings of both pairs of V.
// One thread owns one row; a workgroup owns a tile of 256 consecutive rows of
// one sector; workgroups are persistent and stride over the tile list.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "fh_common.hpp"

namespace fh {

template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

__device__ __forceinline__ int virtual_block(int xcd_order) {
    const int b = blockIdx.x, G = gridDim.x;
    // Workgroups are dealt to the 8 XCDs round robin; map each XCD to a
    // contiguous range of virtual ids so that its L2 sees neighbouring tiles.
    if (xcd_order && (G & 7) == 0) return (b & 7) * (G >> 3) + (b >> 3);
    return b;
}

// The work units (tiles, or passes over tiles) a persistent workgroup walks:
// first, first + step, ... < end.  Workgroups are dealt to the 8 XCDs round
// robin (blockIdx.x mod 8).
//   xcd_order 0: unit b, b + G, ...
//   xcd_order 1: the XCDs take contiguous chunks of G/8 units in turn
//   xcd_order 2: XCD x walks the x-th contiguous eighth of all units, so its
//                L2 sees one sliding neighbourhood of the state vector
//   xcd_order 3: chunks of about G/8 units dealt to the XCDs round robin (as
//                in order 1), each XCD taking its chunks' units in order from a
//                counter of that XCD (queued_unit): the units in flight on an
//                XCD stay one compact run however its workgroups drift, and all
//                XCDs work in one window of the vector, which the memory-side
//                cache shares.  Kernels without counters walk it as order 1.
struct UnitWalk {
    int first, end, step;
};
__device__ __forceinline__ UnitWalk unit_walk(int xcd_order, int nunits) {
    const int b = blockIdx.x, G = gridDim.x;
    if (xcd_order == 2 && (G & 7) == 0) {
        const int x = b & 7;
        const int lo = (int)((long long)nunits * x / 8), hi = (int)((long long)nunits * (x + 1) / 8);
        return UnitWalk{lo + (b >> 3), hi, G >> 3};
    }
    return UnitWalk{virtual_block(xcd_order == 0 ? 0 : 1), nunits, G};
}

// Order 3: the unit of this XCD's k-th ticket (k from its counter, the same
// for the whole workgroup), or nunits when the XCD has none left.  Chunks of K
// units, K the power of two >= G/8 (about one unit per workgroup of the XCD),
// so that the arithmetic is shifts.  Grid a multiple of 8.
__device__ __forceinline__ int queued_unit(int nunits, unsigned k) {
    const unsigned per = gridDim.x >> 3;
    const unsigned L = per <= 1 ? 0u : 32u - (unsigned)__builtin_clz(per - 1u);
    const unsigned long long u = ((((unsigned long long)(k >> L)) * 8u + (blockIdx.x & 7u)) << L) |
                                 (k & ((1u << L) - 1u));
    return u < (unsigned long long)nunits ? (int)u : nunits;
}

template <int M>
__device__ __forceinline__ int modM(int x) {
    x %= M;
    return x < 0 ? x + M : x;
}

template <int M>
constexpr int cmod(int x) {
    return ((x % M) + M) % M;
}

// Table offset of T_s(R_s + dR, Q_s + dQ) relative to the row's key for mode
// s, for a move that adds the modes in 'add' and removes those in 'rem'
// (entries -1 are unused).
template <int M>
constexpr int move_offset(int s, int add0, int add1, int rem0, int rem1) {
    int dR = 0, dQ = 0;
    if (add0 >= 0 && add0 >= s) { dR += 1; dQ += add0; }
    if (add1 >= 0 && add1 >= s) { dR += 1; dQ += add1; }
    if (rem0 >= 0 && rem0 >= s) { dR -= 1; dQ -= rem0; }
    if (rem1 >= 0 && rem1 >= s) { dR -= 1; dQ -= rem1; }
    return (dR + kRBias) * 2 * M + cmod<M>(dQ);
}

// Unrank row r of sector (N, P) with the table in LDS.
//   D_{m+1}(R', Q') = T_{m+2}(R' + 1, Q' + m + 1)     for m + 1 <= M - 2
//   D_{M-1}(R', Q') = [(M - 1) R' == Q' (mod M)]
// With SC > 1 the table holds SC * T and r is SC times the row (unsigned, so
// that sector offsets up to 2^32 stay exact).
template <int M, unsigned SC = 1>
__device__ __forceinline__ void unrank_row(const int* sT, int Rdim, int N, int P, unsigned r, int (&n)[M]) {
    constexpr int P2 = 2 * M;
    int R = N, Q = P;
#pragma unroll
    for (int m = 0; m < M - 1; ++m) {
        int v = 0;
        while (v < R) {
            const int q = modM<M>(Q - m * v);
            unsigned cnt;
            if (m + 1 <= M - 2) {
                cnt = (unsigned)sT[(m + 1) * Rdim * P2 + (R - v + 1 + kRBias) * P2 + modM<M>(q + m + 1)];
            } else {
                cnt = (modM<M>((M - 1) * (R - v)) == q) ? SC : 0u;
            }
            if (r < cnt) break;
            r -= cnt;
            ++v;
        }
        n[m] = v;
        R -= v;
        Q = modM<M>(Q - m * v);
    }
    n[M - 1] = R;
}

// key[s] (s >= 1): table index of T_s at the row's own suffix sums.
// C[x] = sum_{s=1}^{x} T_s(R_s, Q_s), C[0] = 0.
template <int M, typename CT = int>
__device__ __forceinline__ void row_keys(const int* sT, int Rdim, const int (&n)[M], int (&key)[M], CT (&C)[M]) {
    constexpr int P2 = 2 * M;
    int Rs[M], Qs[M];
    int R = 0, Q = 0;
#pragma unroll
    for (int s = M - 1; s >= 1; --s) {
        R += n[s];
        Q = modM<M>(Q + s * n[s]);
        Rs[s] = R;
        Qs[s] = Q;
    }
    C[0] = 0;
    key[0] = 0;
#pragma unroll
    for (int s = 1; s < M; ++s) {
        key[s] = (s - 1) * Rdim * P2 + Rs[s] * P2 + Qs[s];
        C[s] = C[s - 1] + (CT)sT[key[s] + kRBias * P2];
    }
}

// Rank of the neighbour n + e_add0 + e_add1 - e_rem0 - e_rem1 inside the
// sector of dimension dim_dst, given the row's keys (modes lo..hi changed).
template <int M, int LO, int HI, int A0, int A1, int R0, int R1>
__device__ __forceinline__ int move_rank(const int* sT, const int (&key)[M], const int (&C)[M], int dim_dst) {
    // rank' = dim' - 1 - [sum_{s<=LO} T'_s] - [sum_{LO<s<=HI} T'_s] - [sum_{s>HI} T_s]
    int r = dim_dst - 1 - (C[M - 1] - C[HI]);
    static_for<1, HI + 1>([&](auto S) {
        constexpr int s = decltype(S)::value;
        r -= sT[key[s] + move_offset<M>(s, A0, A1, R0, R1)];
    });
    return r;
}

typedef double v2d __attribute__((ext_vector_type(2)));

// Fourth word of a raw buffer resource on gfx9-family GPUs (32-bit data
// format; no swizzle, no stride); out-of-range loads return zero.
constexpr int kBufferWord3 = 0x00020000;

__device__ __forceinline__ v2d nt_load(const double* p) {
    return __builtin_nontemporal_load(reinterpret_cast<const v2d*>(p));
}
__device__ __forceinline__ void nt_store(double* p, v2d v) {
    __builtin_nontemporal_store(v, reinterpret_cast<v2d*>(p));
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum 'NV' per-thread values over the workgroup; thread 0 gets the result in
// out[].  Uses red (>= 4*NV doubles of LDS).
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* red, double* out) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double s = wave_sum(v[q]);
        if (lane == 0) red[wave * NV + q] = s;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double s = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w * NV + threadIdx.x];
        out[threadIdx.x] = s;
    }
    __syncthreads();
}

// Copy the rank table (times SC) and the square-root table into LDS.
template <unsigned SC = 1>
__device__ __forceinline__ void stage_tables(const int* T, int Tn, const double* sq, int nsq, int* sT, double* sSq) {
    for (int q = threadIdx.x; q < Tn; q += blockDim.x) sT[q] = (int)((unsigned)T[q] * SC);
    for (int q = threadIdx.x; q < nsq; q += blockDim.x) sSq[q] = sq[q];
    __syncthreads();
}


// Occupations of a state from its record (occ_stride(M) bytes).
template <int M>
__device__ __forceinline__ void load_occ(const unsigned char* occ, long long state, int (&n)[M]) {
    if constexpr (M <= 8) {
        const uint2 w = reinterpret_cast<const uint2*>(occ)[state];
#pragma unroll
        for (int m = 0; m < M; ++m) n[m] = (int)(((m < 4 ? w.x : w.y) >> (8 * (m & 3))) & 0xffu);
    } else {
        const uint4 w = reinterpret_cast<const uint4*>(occ)[state];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const unsigned v = m < 4 ? w.x : m < 8 ? w.y : m < 12 ? w.z : w.w;
            n[m] = (int)((v >> (8 * (m & 3))) & 0xffu);
        }
    }
}

// ------------------------------------------------------------ H psi stage --
// QUEUE: the variant that takes its units from the per-XCD counters (order 3
// with counters); the static walks are compiled without the counter loop.
template <int M, int NRHS, bool QUEUE>
__global__ __launch_bounds__(kTileRows, stage_min_blocks(M, NRHS)) void stage_kernel(StageArgs A) {
    using CB = Combos<M>;
    constexpr int NP = CB::NP;
    extern __shared__ int smem[];
    int* sT = smem;
    double* sSq = reinterpret_cast<double*>(smem + lds_sqrt_offset(A.Tn));
    // With one right-hand side the rank table is staged times 16, so that
    // neighbour ranks come out directly as byte offsets into the sector.
    constexpr unsigned SC = NRHS == 1 ? 16u : 1u;
    stage_tables<SC>(A.T, A.Tn, A.sqrt_tab, A.nsqrt, sT, sSq);

    // The coefficients are read-only for the whole launch and the same for
    // every lane: read them through the constant address space so that they
    // become scalar loads instead of one vector-memory pass per lane.
    const __attribute__((address_space(4))) double* cf =
        (const __attribute__((address_space(4))) double*)A.coef;
    const double2* X = reinterpret_cast<const double2*>(A.x);
    // With several right-hand sides, G lanes share a row and lane `sub` owns
    // the right-hand sides sub, sub + G, ...: every gather instruction then
    // reads 16*G contiguous bytes per row.  The row's index work is repeated
    // by its G lanes; its cost per right-hand side still falls as 1/NR.  A
    // workgroup then takes one G-th of a tile at a time.
    constexpr int G = stage_lanes_per_row(NRHS);
    constexpr int NR = NRHS / G;
    static_assert(NRHS % G == 0 && kTileRows % G == 0, "lanes per row must divide the tile");
    const int sub = (int)threadIdx.x % G;
    // Tile and sector descriptors are uniform over the workgroup: read them
    // into SGPRs, so that every gather is an SGPR sector base plus a 32-bit
    // lane offset.
    const __attribute__((address_space(4))) Tile* tiles = (const __attribute__((address_space(4))) Tile*)A.tiles;
    const __attribute__((address_space(4))) SecInfo* secs =
        (const __attribute__((address_space(4))) SecInfo*)A.secs;
    const UnitWalk walk = unit_walk(A.xcd_order, A.ntiles * G);
    // Order 3: the next unit comes from this XCD's counter (one vector atomic
    // per workgroup and unit); every workgroup leaves once its XCD has no unit
    // left.
    const bool queued = QUEUE && A.xcd_order == 3 && A.queue != nullptr && (gridDim.x & 7) == 0;
    __shared__ int s_unit;
    for (int vt = walk.first;; vt += walk.step) {
        if (queued) {
            __syncthreads();  // every thread has read the previous unit
            if (threadIdx.x == 0)
                s_unit = queued_unit(walk.end, __hip_atomic_fetch_add(A.queue + (blockIdx.x & 7), 1u,
                                                                      __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
            __syncthreads();
            vt = __builtin_amdgcn_readfirstlane(s_unit);
        }
        if (vt >= walk.end) break;
        const int tsec = __builtin_amdgcn_readfirstlane(tiles[vt / G].sec);
        const int row0 = __builtin_amdgcn_readfirstlane(tiles[vt / G].row0);
        const int nrows = __builtin_amdgcn_readfirstlane(tiles[vt / G].nrows);
        SecInfo sc;
        sc.N = __builtin_amdgcn_readfirstlane(secs[tsec].N);
        sc.P = __builtin_amdgcn_readfirstlane(secs[tsec].P);
        sc.dim = __builtin_amdgcn_readfirstlane(secs[tsec].dim);
        {
            const unsigned long long o = (unsigned long long)secs[tsec].off;
            const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)o);
            const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(o >> 32));
            sc.off = (long long)(((unsigned long long)hi << 32) | lo);
        }
        const int lrow = (vt % G) * (kTileRows / G) + (int)threadIdx.x / G;
        if (lrow >= nrows) continue;
        const int row = row0 + lrow;

        const unsigned rowS = (unsigned)row * SC;
        int n[M];
        unrank_row<M, SC>(sT, A.Rdim, sc.N, sc.P, rowS, n);
        int key[M];
        unsigned C[M];
        row_keys<M, unsigned>(sT, A.Rdim, n, key, C);
        double sq[M], sqp[M];
#pragma unroll
        for (int s = 0; s < M; ++s) {
            sq[s] = sSq[n[s]];
            sqp[s] = sSq[n[s] + 1];
        }
        double diag = 0.0;
#pragma unroll
        for (int s = 0; s < M; ++s) diag = fma(cf[s], (double)n[s], diag);
        static_for<0, NP>([&](auto Pc) {
            constexpr int p = decltype(Pc)::value;
            constexpr int i = CB::pairs.i[p], j = CB::pairs.j[p];
            const double occ = (i == j) ? (double)(n[i] * (n[i] - 1)) : (double)(n[i] * n[j]);
            diag = fma(cf[M + p], occ, diag);
        });

        const long long soff = sc.off;
        const double2* xs = X + soff * NRHS;
        double2 acc[NR];
#pragma unroll
        for (int q = 0; q < NR; ++q) acc[q] = make_double2(0.0, 0.0);

        {
            // One momentum class at a time, in chunks of kGatherBatch / NR
            // combinations: all neighbour ranks first, then every gather of the
            // chunk in flight together, then the FMAs.  For each row pair the
            // source terms W c_kl x are summed first and scaled by c_ij once.
            // Lanes whose row pair cannot be annihilated (c_ij == 0) load zero
            // (one rhs) or their own row (several) and scale it by zero, so the
            // chunk is straight-line code.  Every NRHS sums each column in the
            // same order.
            // One right-hand side: gathers are buffer loads over the sector's
            // bytes.  A lane whose row pair is empty (c_ij == 0) asks for byte
            // kNoGather, past the end of every sector (fewer than 2^28 states),
            // and the load returns zero without a memory access; the term is
            // scaled by c_ij == 0 in any case.
            constexpr unsigned kNoGather = 0xFFFFFF00u;
            const __amdgpu_buffer_rsrc_t xrs = __builtin_amdgcn_make_buffer_rsrc(
                (void*)xs, (short)0, (int)((unsigned)sc.dim * 16u), kBufferWord3);  // bytes, < 2^32
            static_for<0, M>([&](auto Cc) {
                constexpr int c = decltype(Cc)::value;
                constexpr int S = CB::class_size(c);
                if constexpr (S > 1) {
                    constexpr int NQ = S * (S - 1);
                    double cij[S], ckl[S];
                    static_for<0, S>([&](auto R1) {
                        constexpr int r1 = decltype(R1)::value;
                        constexpr int p1 = CB::class_member(c, r1);
                        constexpr int i = CB::pairs.i[p1], j = CB::pairs.j[p1];
                        // as the row pair: sqrt(n_i (n_j - d_ij)), zero exactly
                        // when the pair is empty; as the source pair:
                        // sqrt((n_i + 1)(n_j + 1 + d_ij))
                        if constexpr (i == j) {
                            cij[r1] = sq[i] * sSq[n[i] > 0 ? n[i] - 1 : 0];
                            ckl[r1] = sqp[i] * sSq[n[i] + 2];
                        } else {
                            cij[r1] = sq[i] * sq[j];
                            ckl[r1] = sqp[i] * sqp[j];
                        }
                    });
                    double2 pacc[NR];  // source sum of the current row pair
                    constexpr int QB = kGatherBatch / NR;
                    constexpr int NCH = (NQ + QB - 1) / QB;
                    static_for<0, NCH>([&](auto Ch) {
                        constexpr int q0 = decltype(Ch)::value * QB;
                        constexpr int NQC = (NQ - q0) < QB ? (NQ - q0) : QB;
                        // byte offset (one rhs) or element index (several)
                        using off_t = std::conditional_t<NRHS == 1, unsigned, long long>;
                        off_t off[NQC];
                        static_for<0, NQC>([&](auto Q) {
                            constexpr int q = q0 + decltype(Q)::value;
                            constexpr int r1 = q / (S - 1), t = q % (S - 1), r2 = t < r1 ? t : t + 1;
                            constexpr int p1 = CB::class_member(c, r1), p2 = CB::class_member(c, r2);
                            constexpr int i = CB::pairs.i[p1], j = CB::pairs.j[p1];
                            constexpr int k = CB::pairs.i[p2], l = CB::pairs.j[p2];
                            constexpr int lo = i < k ? i : k;
                            constexpr int hi = j > l ? j : l;
                            unsigned r = rowS + (C[hi] - C[lo]);
                            static_for<lo + 1, hi + 1>([&](auto Sx) {
                                constexpr int s = decltype(Sx)::value;
                                r -= (unsigned)sT[key[s] + move_offset<M>(s, k, l, i, j)];
                            });
                            const unsigned src = cij[r1] != 0.0 ? r : (NRHS == 1 ? kNoGather : rowS);
                            if constexpr (NRHS == 1) off[decltype(Q)::value] = src;
                            else off[decltype(Q)::value] = (long long)src * NRHS + sub;
                        });
                        double2 v[NQC][NR];
                        static_for<0, NQC>([&](auto Q) {
                            if constexpr (NRHS == 1) {
                                v[decltype(Q)::value][0] = __builtin_bit_cast(
                                    double2, __builtin_amdgcn_raw_buffer_load_b128(xrs, off[decltype(Q)::value], 0, 0));
                            } else {
                                const double2* sp = xs + off[decltype(Q)::value];
#pragma unroll
                                for (int j = 0; j < NR; ++j) v[decltype(Q)::value][j] = sp[j * G];
                            }
                        });
                        static_for<0, NQC>([&](auto Q) {
                            constexpr int q = q0 + decltype(Q)::value;
                            constexpr int r1 = q / (S - 1), t = q % (S - 1), r2 = t < r1 ? t : t + 1;
                            constexpr int p1 = CB::class_member(c, r1), p2 = CB::class_member(c, r2);
                            constexpr int ci = M + NP + CB::index(p1, p2);
                            const double w = cf[ci] * ckl[r2];
#pragma unroll
                            for (int j = 0; j < NR; ++j) {
                                const double2 x = v[decltype(Q)::value][j];
                                if constexpr (t == 0) {
                                    pacc[j].x = w * x.x;
                                    pacc[j].y = w * x.y;
                                } else {
                                    pacc[j].x = fma(w, x.x, pacc[j].x);
                                    pacc[j].y = fma(w, x.y, pacc[j].y);
                                }
                                if constexpr (t == S - 2) {
                                    acc[j].x = fma(cij[r1], pacc[j].x, acc[j].x);
                                    acc[j].y = fma(cij[r1], pacc[j].y, acc[j].y);
                                }
                            }
                        });
                        // Keep chunks apart: no table read is reused across them
                        // and the scheduler does not interleave their gathers,
                        // which would otherwise hoist everything and spill.
                        asm volatile("" ::: "memory");
                        __builtin_amdgcn_sched_barrier(0);
                    });
                }
            });
        }
        // Pin the accumulators here: otherwise the compiler sinks each
        // column's FMA chain into the mode branches below (its only users)
        // and keeps every gathered amplitude alive until then.
        if constexpr (NR > 1) {
#pragma unroll
            for (int q = 0; q < NR; ++q) asm volatile("" : "+v"(acc[q].x), "+v"(acc[q].y));
        }

#pragma unroll
        for (int q = 0; q < NR; ++q) {
            const long long e = (soff + row) * NRHS + (NRHS == 1 ? 0 : sub + q * G);
            const double2 xv = X[e];
            double2 h1;
            h1.x = fma(diag, xv.x, acc[q].x);
            h1.y = fma(diag, xv.y, acc[q].y);
            if (A.mode == kApply) {
                reinterpret_cast<double2*>(A.out)[e] = h1;
                continue;
            }
            double2 kk;
            kk.x = A.ks_re * h1.x - A.ks_im * h1.y;
            kk.y = A.ks_re * h1.y + A.ks_im * h1.x;
            // base, acc and baseout are touched once per row per stage: stream
            // them past the caches (non-temporal) so that the gathered vector
            // keeps L2 and the memory-side cache.
            if (A.mode == kLast) {
                const v2d ac = nt_load(A.acc + 2 * e);
                nt_store(A.baseout + 2 * e, v2d{fma(A.a, kk.x, ac.x), fma(A.a, kk.y, ac.y)});
                continue;
            }
            const v2d bs = nt_load(A.base + 2 * e);
            const v2d ac = (A.mode == kFirst) ? bs : nt_load(A.acc + 2 * e);
            nt_store(A.acc + 2 * e, v2d{fma(A.a, kk.x, ac.x), fma(A.a, kk.y, ac.y)});
            reinterpret_cast<double2*>(A.ynext)[e] =
                make_double2(fma(A.b, kk.x, A.c0 * bs.x), fma(A.b, kk.y, A.c0 * bs.y));
        }
    }
}

// ---------------------------------------------------------------- moments --
// group 0: [0] <psi|psi>, [1+i] <a_i>, [1+M+i] <a_i^+ a_i>
// group 1+i: [j] <a_i^+ a_j> (j != i), [M+l] <a_i a_l> (l >= i)
// Each term: sum_n conj(psi(n')) c psi(n) with n' the image of n.  Rows start
// from their occupation records; tile, sector and sector-map entries are
// uniform per workgroup and read with scalar loads.
template <int M>
__global__ __launch_bounds__(kTileRows) void moments_kernel(MomArgs A) {
    constexpr int NO = momentsOut(M);
    using C4 = const __attribute__((address_space(4))) int;
    extern __shared__ int smem[];
    int* sT = smem;
    double* sSq = reinterpret_cast<double*>(smem + lds_sqrt_offset(A.Tn));
    double* red = sSq + A.nsqrt;
    stage_tables(A.T, A.Tn, A.sqrt_tab, A.nsqrt, sT, sSq);

    const double2* __restrict__ X = reinterpret_cast<const double2*>(A.psi);
    const __attribute__((address_space(4))) Tile* tiles = (const __attribute__((address_space(4))) Tile*)A.tiles;
    const __attribute__((address_space(4))) SecInfo* secs =
        (const __attribute__((address_space(4))) SecInfo*)A.secs;
    C4* secmap = (C4*)A.secmap;
    const int g = blockIdx.y;
    const int nrhs = A.nrhs, rhs = A.rhs;
    double acc[2 * NO];
#pragma unroll
    for (int q = 0; q < 2 * NO; ++q) acc[q] = 0.0;

    auto add = [&](int slot, double2 y, double c, double2 x) {
        // conj(y) * c * x
        acc[2 * slot] = fma(c, y.x * x.x + y.y * x.y, acc[2 * slot]);
        acc[2 * slot + 1] = fma(c, y.x * x.y - y.y * x.x, acc[2 * slot + 1]);
    };
    // partner sector (N2, P2): its dimension and offset, false if absent
    auto partner = [&](int N2, int P2, int& dim, long long& off) -> bool {
        const int sid = __builtin_amdgcn_readfirstlane(secmap[N2 * M + P2]);
        if (sid < 0) return false;
        dim = __builtin_amdgcn_readfirstlane(secs[sid].dim);
        const unsigned long long o = (unsigned long long)secs[sid].off;
        off = (long long)(((unsigned long long)__builtin_amdgcn_readfirstlane((unsigned)(o >> 32)) << 32) |
                          __builtin_amdgcn_readfirstlane((unsigned)o));
        return true;
    };

    const UnitWalk walk = unit_walk(A.xcd_order, A.ntiles);
    for (int t = walk.first; t < walk.end; t += walk.step) {
        const int tsec = __builtin_amdgcn_readfirstlane(tiles[t].sec);
        const int row0 = __builtin_amdgcn_readfirstlane(tiles[t].row0);
        const int nrows = __builtin_amdgcn_readfirstlane(tiles[t].nrows);
        const int N = __builtin_amdgcn_readfirstlane(secs[tsec].N);
        const int P = __builtin_amdgcn_readfirstlane(secs[tsec].P);
        const long long soff = secs[tsec].off;
        if ((int)threadIdx.x >= nrows) continue;
        const int row = row0 + (int)threadIdx.x;
        int n[M];
        load_occ<M>(A.occ, soff + row, n);
        int key[M], C[M];
        row_keys<M>(sT, A.Rdim, n, key, C);
        const double2 x = X[(soff + row) * nrhs + rhs];
        if (g == 0) {
            const double x2 = x.x * x.x + x.y * x.y;
            acc[0] += x2;
            static_for<0, M>([&](auto I) {
                constexpr int i = decltype(I)::value;
                acc[2 * (1 + M + i)] = fma((double)n[i], x2, acc[2 * (1 + M + i)]);
                int pdim;
                long long poff;
                if (N >= 1 && partner(N - 1, modM<M>(P - i), pdim, poff) && n[i] >= 1) {
                    const int r = move_rank<M, 0, i, -1, -1, i, -1>(sT, key, C, pdim);
                    add(1 + i, X[(poff + r) * nrhs + rhs], sSq[n[i]], x);
                }
            });
        } else {
            static_for<0, M>([&](auto I) {
                constexpr int i = decltype(I)::value;
                if (g == 1 + i) {
                    // <a_i^+ a_j>: n' = n - e_j + e_i, c = sqrt(n_j (n_i + 1))
                    static_for<0, M>([&](auto J) {
                        constexpr int j = decltype(J)::value;
                        if constexpr (j != i) {
                            int pdim;
                            long long poff;
                            if (partner(N, modM<M>(P + i - j), pdim, poff) && n[j] >= 1) {
                                constexpr int hi = i > j ? i : j;
                                const int r = move_rank<M, 0, hi, i, -1, j, -1>(sT, key, C, pdim);
                                add(j, X[(poff + r) * nrhs + rhs], sSq[n[j]] * sSq[n[i] + 1], x);
                            }
                        }
                    });
                    // <a_i a_l>, l >= i: n' = n - e_i - e_l, c = sqrt(n_l (n_i - d_il))
                    static_for<i, M>([&](auto L) {
                        constexpr int l = decltype(L)::value;
                        const bool ok = (l == i) ? (n[i] >= 2) : (n[i] >= 1 && n[l] >= 1);
                        int pdim;
                        long long poff;
                        if (N >= 2 && partner(N - 2, modM<M>(P - i - l), pdim, poff) && ok) {
                            const int r = move_rank<M, 0, l, -1, -1, i, l>(sT, key, C, pdim);
                            const double c = (l == i) ? sSq[n[i]] * sSq[n[i] - 1] : sSq[n[l]] * sSq[n[i]];
                            add(M + l, X[(poff + r) * nrhs + rhs], c, x);
                        }
                    });
                }
            });
        }
    }
    __shared__ double outv[2 * kMomOutMax];
    block_sum<2 * NO>(acc, red, outv);
    if (threadIdx.x < 2 * NO) {
        A.partial[((size_t)g * gridDim.x + blockIdx.x) * 2 * kMomOutMax + threadIdx.x] = outv[threadIdx.x];
    }
}

// ------------------------------------------------------- one-body source --
template <int M>
__global__ __launch_bounds__(kTileRows) void onebody_kernel(OneBodyArgs A) {
    extern __shared__ int smem[];
    int* sT = smem;
    double* sSq = reinterpret_cast<double*>(smem + lds_sqrt_offset(A.Tn));
    stage_tables(A.T, A.Tn, A.sqrt_tab, A.nsqrt, sT, sSq);
    const double2* __restrict__ X = reinterpret_cast<const double2*>(A.psi);
    const double* cf = A.cf;
    const int nrhs = A.nrhs, rhs = A.rhs;
    for (int t = blockIdx.x; t < A.ntiles; t += gridDim.x) {
        const Tile tl = A.tiles[t];
        if ((int)threadIdx.x >= tl.nrows) continue;
        const SecInfo sc = A.secs[tl.sec];
        const int row = tl.row0 + (int)threadIdx.x;
        int n[M];
        unrank_row<M>(sT, A.Rdim, sc.N, sc.P, row, n);
        int key[M], C[M];
        row_keys<M>(sT, A.Rdim, n, key, C);
        const int N = sc.N, P = sc.P;
        const double2 x = X[(sc.off + row) * nrhs + rhs];
        double ox = 0.0, oy = 0.0;
        auto cmul_add = [&](double cr, double ci, double s, double2 y) {
            // (cr + i ci) * s * y
            ox += s * (cr * y.x - ci * y.y);
            oy += s * (cr * y.y + ci * y.x);
        };
        double nt = 0.0;
#pragma unroll
        for (int s = 0; s < M; ++s) nt += (double)n[s];
        cmul_add(cf[0] + cf[2] * nt, cf[1] + cf[3] * nt, 1.0, x);
        static_for<0, M>([&](auto I) {
            constexpr int i = decltype(I)::value;
            const double* u = cf + 4 + 2 * i;
            const double* v = cf + 4 + 2 * M + 2 * i;
            // (a_i x)(n) = sqrt(n_i + 1) x(n + e_i)
            if (N + 1 <= A.Nmax) {
                const int sid = A.secmap[(N + 1) * M + modM<M>(P + i)];
                if (sid >= 0) {
                    const SecInfo pd = A.secs[sid];
                    const int r = move_rank<M, 0, i, i, -1, -1, -1>(sT, key, C, pd.dim);
                    cmul_add(u[0], u[1], sSq[n[i] + 1], X[(pd.off + r) * nrhs + rhs]);
                }
            }
            // (a_i^+ x)(n) = sqrt(n_i) x(n - e_i)
            if (N >= 1 && n[i] >= 1) {
                const int sid = A.secmap[(N - 1) * M + modM<M>(P - i)];
                if (sid >= 0) {
                    const SecInfo pd = A.secs[sid];
                    const int r = move_rank<M, 0, i, -1, -1, i, -1>(sT, key, C, pd.dim);
                    cmul_add(v[0], v[1], sSq[n[i]], X[(pd.off + r) * nrhs + rhs]);
                }
            }
            static_for<0, M>([&](auto J) {
                constexpr int j = decltype(J)::value;
                const double* h = cf + 4 + 4 * M + 2 * (i * M + j);
                if constexpr (i == j) {
                    cmul_add(h[0], h[1], (double)n[i], x);
                } else {
                    // (a_i^+ a_j x)(n) = sqrt(n_i (n_j + 1)) x(n - e_i + e_j)
                    if (n[i] >= 1) {
                        const int sid = A.secmap[N * M + modM<M>(P - i + j)];
                        if (sid >= 0) {
                            const SecInfo pd = A.secs[sid];
                            constexpr int hi = i > j ? i : j;
                            const int r = move_rank<M, 0, hi, j, -1, i, -1>(sT, key, C, pd.dim);
                            cmul_add(h[0], h[1], sSq[n[i]] * sSq[n[j] + 1], X[(pd.off + r) * nrhs + rhs]);
                        }
                    }
                }
            });
        });
        reinterpret_cast<double2*>(A.out)[(sc.off + row) * nrhs + rhs] = make_double2(ox, oy);
    }
}

// ------------------------------------------------------- correlators -----
// Fill the occupation records of every state (unrank once per state).
template <int M>
__global__ __launch_bounds__(kTileRows) void occ_table_kernel(OccArgs A) {
    extern __shared__ int smem[];
    int* sT = smem;
    for (int q = threadIdx.x; q < A.Tn; q += blockDim.x) sT[q] = A.T[q];
    __syncthreads();
    for (int t = blockIdx.x; t < A.ntiles; t += gridDim.x) {
        const Tile tl = A.tiles[t];
        if ((int)threadIdx.x >= tl.nrows) continue;
        const SecInfo sc = A.secs[tl.sec];
        const int row = tl.row0 + (int)threadIdx.x;
        int n[M];
        unrank_row<M>(sT, A.Rdim, sc.N, sc.P, row, n);
        unsigned w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int m = 0; m < M; ++m) w[m >> 2] |= (unsigned)n[m] << (8 * (m & 3));
        const long long state = sc.off + row;
        if constexpr (M <= 8) reinterpret_cast<uint2*>(A.occ)[state] = make_uint2(w[0], w[1]);
        else reinterpret_cast<uint4*>(A.occ)[state] = make_uint4(w[0], w[1], w[2], w[3]);
    }
}

// G[r1 * S + r2] += sum_q sum_n conj(uscale_q u_q(n)) <n| a_i^+ a_j^+ a_k a_l |n'> y_q(n')
// for the pairs p1 = member(C, r1) = {i,j}, p2 = member(C, r2) = {k,l} of one
// momentum class C, n' = n - e_i - e_j + e_k + e_l (n' = n when r1 == r2),
// over the kCorrPairs vector pairs (u_q, y_q).  The pairs share the row's setup
// and every neighbour rank; their terms go into the same sums.  One body per
// class keeps exactly that class's S^2 complex sums in registers across the
// persistent tile loop; rows start from their occupation records.  Partials
// are written with row stride max_class_size.  With one right-hand side
// (SC = 16) the rank table is staged times 16, neighbour ranks come out as
// byte offsets into the sector, and the gathers are buffer loads from an
// SGPR sector base (empty row pairs load zero from past the end, as in the
// stage kernel); tile and sector descriptors are scalar loads.
template <int M, int C, unsigned SC>
__device__ __forceinline__ void corr_class(const CorrArgs& A) {
    using CB = Combos<M>;
    constexpr int S = CB::class_size(C);
    constexpr int SMAX = CB::max_class_size();
    // Only the imaginary parts are summed: with V real, dJ/dV and dJ/dLambda
    // need Im <u|X|y> alone.  One double per pair of pairs.
    constexpr int NV = S * S;
    constexpr int NPR = corr_pairs_per_launch(M);  // the launch's pairs are u[0..NPR), y[0..NPR)
    extern __shared__ int smem[];
    int* sT = smem;
    double* sSq = reinterpret_cast<double*>(smem + lds_sqrt_offset(A.Tn));
    double* red = sSq + A.nsqrt;
    stage_tables<SC>(A.T, A.Tn, A.sqrt_tab, A.nsqrt, sT, sSq);
    const int nrhs = SC == 16 ? 1 : A.nrhs, rhs = SC == 16 ? 0 : A.rhs;
    double acc[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) acc[q] = 0.0;
    // Im(conj(u) y) summed over the pairs
    auto cdot_im = [](const double2 (&u)[NPR], const double2 (&y)[NPR]) {
        double ti = 0.0;
#pragma unroll
        for (int p = 0; p < NPR; ++p) ti = fma(u[p].x, y[p].y, fma(-u[p].y, y[p].x, ti));
        return ti;
    };
    const __attribute__((address_space(4))) Tile* tiles = (const __attribute__((address_space(4))) Tile*)A.tiles;
    const __attribute__((address_space(4))) SecInfo* secs =
        (const __attribute__((address_space(4))) SecInfo*)A.secs;
    const UnitWalk walk = unit_walk(A.xcd_order, A.ntiles);
    // Order 3: this class's workgroups on an XCD take its tiles in order from
    // the counter of (class, XCD), as in the stage kernel.  Not at M >= 8, where
    // the class's sums fill the registers and the queue's barriers made the
    // compiler spill (108 B per lane at M = 8, 440 B at M = 10); there the walk
    // is order 2.
    constexpr bool kQueue = M <= 7;
    const bool queued = kQueue && A.xcd_order == 3 && A.queue != nullptr && (gridDim.x & 7) == 0;
    __shared__ unsigned s_ticket;
    for (int t = walk.first;; t += walk.step) {
        if (queued) {
            __syncthreads();  // every thread has read the previous ticket
            if (threadIdx.x == 0)
                s_ticket = __hip_atomic_fetch_add(A.queue + 8 * C + (blockIdx.x & 7), 1u, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
            __syncthreads();
            t = queued_unit(walk.end, __builtin_amdgcn_readfirstlane(s_ticket));
        }
        if (t >= walk.end) break;
        const int tsec = __builtin_amdgcn_readfirstlane(tiles[t].sec);
        const int row0 = __builtin_amdgcn_readfirstlane(tiles[t].row0);
        const int nrows = __builtin_amdgcn_readfirstlane(tiles[t].nrows);
        if ((int)threadIdx.x >= nrows) continue;
        const unsigned dim = (unsigned)__builtin_amdgcn_readfirstlane(secs[tsec].dim);
        long long soff;
        {
            const unsigned long long o = (unsigned long long)secs[tsec].off;
            const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)o);
            const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(o >> 32));
            soff = (long long)(((unsigned long long)hi << 32) | lo);
        }
        const int row = row0 + (int)threadIdx.x;
        const long long state = soff + row;
        const unsigned rowS = (unsigned)row * SC;
        int n[M];
        load_occ<M>(A.occ, state, n);
        int key[M];
        unsigned Cs[M];
        row_keys<M, unsigned>(sT, A.Rdim, n, key, Cs);
        double2 u[NPR], y0[NPR];
#pragma unroll
        for (int p = 0; p < NPR; ++p) {
            u[p] = reinterpret_cast<const double2*>(A.u[p])[state * nrhs + rhs];
            u[p].x *= A.uscale[p];
            u[p].y *= A.uscale[p];
            y0[p] = reinterpret_cast<const double2*>(A.y[p])[state * nrhs + rhs];
        }
        double cij[S], ckl[S];
        static_for<0, S>([&](auto R1) {
            constexpr int r1 = decltype(R1)::value;
            constexpr int p1 = CB::class_member(C, r1);
            constexpr int i = CB::pairs.i[p1], j = CB::pairs.j[p1];
            if constexpr (i == j) {
                cij[r1] = sSq[n[i]] * sSq[n[i] > 0 ? n[i] - 1 : 0];
                ckl[r1] = sSq[n[i] + 1] * sSq[n[i] + 2];
            } else {
                cij[r1] = sSq[n[i]] * sSq[n[j]];
                ckl[r1] = sSq[n[i] + 1] * sSq[n[j] + 1];
            }
        });
        {
            // p1 == p2: <n|a_i^+ a_j^+ a_i a_j|n> = c_ij^2
            const double ti = cdot_im(u, y0);
            static_for<0, S>([&](auto R1) {
                constexpr int r1 = decltype(R1)::value;
                constexpr int o = r1 * S + r1;
                acc[o] = fma(cij[r1] * cij[r1], ti, acc[o]);
            });
        }
        if constexpr (S > 1) {
            // Off-diagonal pairs in chunks: neighbour ranks (shared by the
            // vector pairs), then the gathers in flight together, then the sums.
            // Lanes whose row pair is empty (c_ij == 0) gather their own row
            // and add zero.
            constexpr int NQ = S * (S - 1);
            constexpr int QB = S >= 5 ? kGatherBatch / (2 * NPR) : kGatherBatch / NPR;
            constexpr int NCH = (NQ + QB - 1) / QB;
            constexpr unsigned kNoGather = 0xFFFFFF00u;
            __amdgpu_buffer_rsrc_t yrs[NPR];
            if constexpr (SC == 16) {
#pragma unroll
                for (int p = 0; p < NPR; ++p)
                    yrs[p] = __builtin_amdgcn_make_buffer_rsrc(
                        (void*)(reinterpret_cast<const double2*>(A.y[p]) + soff), (short)0, (int)(dim * 16u),
                        kBufferWord3);  // bytes, < 2^32
            }
            static_for<0, NCH>([&](auto Ch) {
                constexpr int q0 = decltype(Ch)::value * QB;
                constexpr int NQC = (NQ - q0) < QB ? (NQ - q0) : QB;
                using off_t = std::conditional_t<SC == 16, unsigned, long long>;
                off_t off[NQC];
                static_for<0, NQC>([&](auto Q) {
                    constexpr int q = q0 + decltype(Q)::value;
                    constexpr int r1 = q / (S - 1), tq = q % (S - 1), r2 = tq < r1 ? tq : tq + 1;
                    constexpr int p1 = CB::class_member(C, r1), p2 = CB::class_member(C, r2);
                    constexpr int i = CB::pairs.i[p1], j = CB::pairs.j[p1];
                    constexpr int k = CB::pairs.i[p2], l = CB::pairs.j[p2];
                    constexpr int lo = i < k ? i : k;
                    constexpr int hi = j > l ? j : l;
                    unsigned r = rowS + (Cs[hi] - Cs[lo]);
                    static_for<lo + 1, hi + 1>([&](auto Sx) {
                        constexpr int s2 = decltype(Sx)::value;
                        r -= (unsigned)sT[key[s2] + move_offset<M>(s2, k, l, i, j)];
                    });
                    if constexpr (SC == 16) {
                        off[decltype(Q)::value] = cij[r1] != 0.0 ? r : kNoGather;
                    } else {
                        const int src = cij[r1] != 0.0 ? (int)r : row;
                        off[decltype(Q)::value] = (soff + src) * nrhs + rhs;
                    }
                });
                double2 v[NQC][NPR];
                static_for<0, NQC>([&](auto Q) {
#pragma unroll
                    for (int p = 0; p < NPR; ++p) {
                        if constexpr (SC == 16)
                            v[decltype(Q)::value][p] = __builtin_bit_cast(
                                double2, __builtin_amdgcn_raw_buffer_load_b128(yrs[p], off[decltype(Q)::value], 0, 0));
                        else
                            v[decltype(Q)::value][p] =
                                reinterpret_cast<const double2*>(A.y[p])[off[decltype(Q)::value]];
                    }
                });
                static_for<0, NQC>([&](auto Q) {
                    constexpr int q = q0 + decltype(Q)::value;
                    constexpr int r1 = q / (S - 1), tq = q % (S - 1), r2 = tq < r1 ? tq : tq + 1;
                    constexpr int o = r1 * S + r2;
                    acc[o] = fma(cij[r1] * ckl[r2], cdot_im(u, v[decltype(Q)::value]), acc[o]);
                });
                asm volatile("" ::: "memory");
                __builtin_amdgcn_sched_barrier(0);
            });
        }
    }
    __shared__ double outv[NV];
    block_sum<NV>(acc, red, outv);
    if ((int)threadIdx.x < 2 * kCorrOutMax) {
        const int part = threadIdx.x & 1, slot = threadIdx.x >> 1;
        const int r1 = slot / SMAX, r2 = slot % SMAX;
        const double v = (part == 1 && r1 < S && r2 < S) ? outv[r1 * S + r2] : 0.0;  // real parts: 0
        A.partial[((size_t)C * gridDim.x + blockIdx.x) * 2 * kCorrOutMax + threadIdx.x] = v;
    }
}

// All classes in one launch: blockIdx.y selects the class.  The branch is
// uniform over the workgroup and each class body holds its own sums, so the
// registers are those of the largest class, not of all of them.
template <int M>
__global__ __launch_bounds__(kTileRows, 2) void corr_kernel(CorrArgs A) {
    static_for<0, M>([&](auto Cc) {
        constexpr int c = decltype(Cc)::value;
        if ((int)blockIdx.y == c) {
            if (A.nrhs == 1) corr_class<M, c, 16u>(A);
            else corr_class<M, c, 1u>(A);
        }
    });
}

// ------------------------------------------------------- initial states --
template <int M>
__global__ __launch_bounds__(kTileRows) void init_product_kernel(InitArgs A) {
    extern __shared__ int smem[];
    int* sT = smem;
    for (int q = threadIdx.x; q < A.Tn; q += blockDim.x) sT[q] = A.T[q];
    __syncthreads();
    const double2* tab = reinterpret_cast<const double2*>(A.tab);
    const int W = A.Nmax + 1;
    for (int t = blockIdx.x; t < A.ntiles; t += gridDim.x) {
        const Tile tl = A.tiles[t];
        if ((int)threadIdx.x >= tl.nrows) continue;
        const SecInfo sc = A.secs[tl.sec];
        const int row = tl.row0 + (int)threadIdx.x;
        int n[M];
        unrank_row<M>(sT, A.Rdim, sc.N, sc.P, row, n);
        for (int q = 0; q < A.nrhs; ++q) {
            double2 p = tab[(size_t)(q * M + 0) * W + n[0]];
#pragma unroll
            for (int m = 1; m < M; ++m) {
                const double2 f = tab[(size_t)(q * M + m) * W + n[m]];
                p = make_double2(p.x * f.x - p.y * f.y, p.x * f.y + p.y * f.x);
            }
            reinterpret_cast<double2*>(A.psi)[(sc.off + row) * A.nrhs + q] = p;
        }
    }
}

// S0 = sum conj(g) psi0 ; S_k = sum conj(g) psi0^(k) (factor k from tabd)
template <int M>
__global__ __launch_bounds__(kTileRows) void vjp_kernel(VjpArgs A) {
    constexpr int NV = 2 * (M + 1);
    extern __shared__ int smem[];
    int* sT = smem;
    double* red = reinterpret_cast<double*>(smem + lds_sqrt_offset(A.Tn));
    for (int q = threadIdx.x; q < A.Tn; q += blockDim.x) sT[q] = A.T[q];
    __syncthreads();
    const double2* tab = reinterpret_cast<const double2*>(A.tab);
    const double2* tabd = reinterpret_cast<const double2*>(A.tabd);
    const double2* G = reinterpret_cast<const double2*>(A.g);
    const int W = A.Nmax + 1;
    double acc[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) acc[q] = 0.0;
    for (int t = blockIdx.x; t < A.ntiles; t += gridDim.x) {
        const Tile tl = A.tiles[t];
        if ((int)threadIdx.x >= tl.nrows) continue;
        const SecInfo sc = A.secs[tl.sec];
        const int row = tl.row0 + (int)threadIdx.x;
        int n[M];
        unrank_row<M>(sT, A.Rdim, sc.N, sc.P, row, n);
        const double2 g = G[(sc.off + row) * A.nrhs + A.rhs];
        double2 f[M];
#pragma unroll
        for (int m = 0; m < M; ++m) f[m] = tab[(size_t)m * W + n[m]];
#pragma unroll
        for (int k = -1; k < M; ++k) {
            double2 p = make_double2(1.0, 0.0);
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const double2 fm = (m == k) ? tabd[(size_t)m * W + n[m]] : f[m];
                p = make_double2(p.x * fm.x - p.y * fm.y, p.x * fm.y + p.y * fm.x);
            }
            // conj(g) p
            acc[2 * (k + 1)] += g.x * p.x + g.y * p.y;
            acc[2 * (k + 1) + 1] += g.x * p.y - g.y * p.x;
        }
    }
    __shared__ double outv[2 * (kMaxM + 1)];
    block_sum<NV>(acc, red, outv);
    if (threadIdx.x < NV) A.partial[(size_t)blockIdx.x * 2 * (kMaxM + 1) + threadIdx.x] = outv[threadIdx.x];
}

// ------------------------------------------------------- classical field --
// Mean-field equations of the model (Sec. II, Eq. clEqnMotion; Sec. III.A,
// Eq. classicalFieldEqns): the Heisenberg equation of a_p with operators
// replaced by their means,
//   d alpha_p/dt = -i [ w_p alpha_p + sum_{j,k} U[p][j][k] conj(alpha_j) alpha_k alpha_l ],
//   l = p + j - k (mod M),  U[p][j][k] = (Lambda/2)(V_pjkl + V_jpkl)
// (only momentum-conserving V entries exist).  One thread per trajectory,
// every RK4 step of the run in one launch; coefficients are scalar loads.
template <int M>
__device__ __forceinline__ void classical_rhs(const __attribute__((address_space(4))) double* w,
                                              const __attribute__((address_space(4))) double* U,
                                              const double2 (&y)[M], double2 (&f)[M]) {
    static_for<0, M>([&](auto Pp) {
        constexpr int p = decltype(Pp)::value;
        double sr = 0.0, si = 0.0;
        static_for<0, M>([&](auto Jj) {
            constexpr int j = decltype(Jj)::value;
            double rr = 0.0, ri = 0.0;  // sum_k U y_k y_l
            static_for<0, M>([&](auto Kk) {
                constexpr int k0 = decltype(Kk)::value;
                constexpr int l0 = cmod<M>(p + j - k0);
                constexpr int k = k0 < l0 ? k0 : l0, l = k0 < l0 ? l0 : k0;  // one product per pair
                const double u = U[(p * M + j) * M + k0];
                const double pr = y[k].x * y[l].x - y[k].y * y[l].y;
                const double pi = y[k].x * y[l].y + y[k].y * y[l].x;
                rr = fma(u, pr, rr);
                ri = fma(u, pi, ri);
            });
            sr = fma(y[j].x, rr, fma(y[j].y, ri, sr));   // Re conj(y_j) R
            si = fma(y[j].x, ri, fma(-y[j].y, rr, si));  // Im conj(y_j) R
        });
        const double xr = fma(w[p], y[p].x, sr), xi = fma(w[p], y[p].y, si);
        f[p] = make_double2(xi, -xr);  // -i (xr + i xi)
    });
}

template <int M>
__global__ __launch_bounds__(256) void classical_kernel(ClassicalArgs A) {
    const int tr = blockIdx.x * blockDim.x + threadIdx.x;
    if (tr >= A.ntraj) return;
    using CD = const __attribute__((address_space(4))) double;
    CD* w = (CD*)A.omega;
    CD* U = (CD*)A.U;
    double2* alpha = reinterpret_cast<double2*>(A.alpha);
    double2* out = reinterpret_cast<double2*>(A.out);
    const double dt = A.dt, h2 = 0.5 * A.dt, h6 = A.dt / 6.0;
    double2 y[M];
#pragma unroll
    for (int p = 0; p < M; ++p) y[p] = alpha[(long long)tr * M + p];
    for (long long s = 0;; ++s) {
        if (out && s % A.every == 0) {
            const long long o = ((s / A.every) * A.ntraj + tr) * M;
#pragma unroll
            for (int p = 0; p < M; ++p) out[o + p] = y[p];
        }
        if (s == A.nsteps) break;
        double2 k[M], acc[M], t[M];
        classical_rhs<M>(w, U, y, k);  // k1
#pragma unroll
        for (int p = 0; p < M; ++p) {
            acc[p] = k[p];
            t[p] = make_double2(fma(h2, k[p].x, y[p].x), fma(h2, k[p].y, y[p].y));
        }
        classical_rhs<M>(w, U, t, k);  // k2
#pragma unroll
        for (int p = 0; p < M; ++p) {
            acc[p] = make_double2(fma(2.0, k[p].x, acc[p].x), fma(2.0, k[p].y, acc[p].y));
            t[p] = make_double2(fma(h2, k[p].x, y[p].x), fma(h2, k[p].y, y[p].y));
        }
        classical_rhs<M>(w, U, t, k);  // k3
#pragma unroll
        for (int p = 0; p < M; ++p) {
            acc[p] = make_double2(fma(2.0, k[p].x, acc[p].x), fma(2.0, k[p].y, acc[p].y));
            t[p] = make_double2(fma(dt, k[p].x, y[p].x), fma(dt, k[p].y, y[p].y));
        }
        classical_rhs<M>(w, U, t, k);  // k4
#pragma unroll
        for (int p = 0; p < M; ++p) {
            y[p].x = fma(h6, acc[p].x + k[p].x, y[p].x);
            y[p].y = fma(h6, acc[p].y + k[p].y, y[p].y);
        }
    }
#pragma unroll
    for (int p = 0; p < M; ++p) alpha[(long long)tr * M + p] = y[p];
}

// ------------------------------------------------------ rank / unrank -----
template <int M>
__global__ void rank_kernel(RankArgs A) {
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= A.count) return;
    constexpr int P2 = 2 * M;
    int n[M];
    int N = 0, mom = 0;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        n[m] = A.occ[q * M + m];
        N += n[m];
        mom = modM<M>(mom + m * n[m]);
    }
    if (N != A.N || mom != A.P) {
        A.idx[q] = -1;
        return;
    }
    long long r = (long long)A.dim - 1;
    int R = 0, Q = 0;
#pragma unroll
    for (int s = M - 1; s >= 1; --s) {
        R += n[s];
        Q = modM<M>(Q + s * n[s]);
        r -= A.T[(s - 1) * A.Rdim * P2 + (R + kRBias) * P2 + Q];
    }
    A.idx[q] = r;
}

template <int M>
__global__ void unrank_kernel(RankArgs A) {
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= A.count) return;
    const long long r = A.idx_in[q];
    int n[M];
    if (r < 0 || r >= A.dim) {
#pragma unroll
        for (int m = 0; m < M; ++m) A.occ_out[q * M + m] = 0xff;
        return;
    }
    unrank_row<M>(A.T, A.Rdim, A.N, A.P, (int)r, n);
#pragma unroll
    for (int m = 0; m < M; ++m) A.occ_out[q * M + m] = (uint8_t)n[m];
}

}  // namespace fh

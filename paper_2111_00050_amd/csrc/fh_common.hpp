// fh_common.hpp -- definitions shared by the host code and the gfx950 kernels.
//
// Notation (Sec. II.A, Eq. Ham; Sec. III.B):
//   modes j = 0..M-1, momentum modulus p = M, sector (N, P) = all occupation
//   vectors n with sum n_j = N and sum j n_j == P (mod M).
//
// Pairs.  An unordered mode pair {i, j} (i <= j) is indexed in the order
// (0,0), (0,1), ..., (0,M-1), (1,1), ...  Its class is (i + j) mod M.  The
// interaction a_i^+ a_j^+ a_k a_l conserves momentum iff {i,j} and {k,l} share
// a class, and two different pairs of one class are disjoint, so a nonzero
// off-diagonal matrix element <n| a_i^+ a_j^+ a_k a_l |n'> links
//   n' = n - e_i - e_j + e_k + e_l      ("row pair" {i,j}, "source pair" {k,l})
// and the pair of pairs is unique for every neighbour n' of n.
//
// Combinations.  The off-diagonal combinations are the ordered pairs
// (row pair, source pair) of distinct pairs in one class, enumerated with the
// row pair outermost, both in pair order.  Host and device share this
// enumeration (the coefficient table is laid out in it).
#pragma once
#include <cstdint>

#ifndef __HIPCC__
#define FH_HD
#else
#define FH_HD __host__ __device__
#endif

namespace fh {

constexpr int kMaxM = 10;
constexpr int kTileRows = 256;  // one row per thread, four wave64s per workgroup
constexpr int kRBias = 2;       // rank table rows R = -2 .. Nmax+2
constexpr int kGatherBatch = 16;  // neighbour gathers issued together per thread
// Lanes of the stage kernel that share one row when several right-hand sides
// are evolved together; a workgroup then covers a tile in that many passes.
constexpr FH_HD int stage_lanes_per_row(int nrhs) { return nrhs >= 4 ? 4 : nrhs; }
#ifndef FH_STAGE_BLOCKS_PER_CU
#define FH_STAGE_BLOCKS_PER_CU 1
#endif
// Occupancy target of the stage kernel (workgroups of 256 per CU); it caps the
// registers per thread at 512 / (4 * blocks) per SIMD lane.
constexpr int kStageBlocksPerCU = FH_STAGE_BLOCKS_PER_CU;
// Minimum workgroups per CU the one-column stage kernel is compiled for: the
// occupancy its register count reaches without the tile-queue loop (M <= 3:
// 8 waves per SIMD; M = 4: <= 80 VGPRs, 6; M = 5: <= 96, 5; M = 6: <= 128, 4;
// M = 7, 8: <= 168, 3; M >= 9: 2), so that the queue's few extra registers do
// not cost a wave per SIMD.  Several columns: no bound (the 16-column kernel
// holds 256 VGPRs at one wave).
// The stage kernel's counter walk (XCD order 3) pays from M = 7 on; at M <= 6
// (54 gathers per row or fewer) the static walk of order 1 is faster (M = 6:
// 4.20 against 4.66 ms per H psi on 55.5M states), and the counter variant is
// not built.
constexpr int kStageCounterMinM = 7;
constexpr FH_HD int stage_min_blocks(int M, int nrhs) {
    return nrhs > 1 ? kStageBlocksPerCU : (M <= 3 ? 8 : M == 4 ? 6 : M == 5 ? 5 : M == 6 ? 4 : M <= 8 ? 3 : 2);
}

template <int M>
struct PairTable {
    static constexpr int NP = M * (M + 1) / 2;
    int i[NP];
    int j[NP];
    constexpr PairTable() : i{}, j{} {
        int c = 0;
        for (int a = 0; a < M; ++a)
            for (int b = a; b < M; ++b) {
                i[c] = a;
                j[c] = b;
                ++c;
            }
    }
};

template <int M>
struct Combos {
    static constexpr int NP = M * (M + 1) / 2;
    static constexpr PairTable<M> pairs{};
    static constexpr int cls(int p) { return (pairs.i[p] + pairs.j[p]) % M; }
    static constexpr bool linked(int p1, int p2) { return p1 != p2 && cls(p1) == cls(p2); }
    static constexpr int count() {
        int c = 0;
        for (int p1 = 0; p1 < NP; ++p1)
            for (int p2 = 0; p2 < NP; ++p2)
                if (linked(p1, p2)) ++c;
        return c;
    }
    static constexpr int NC = count();
    static constexpr int index(int p1, int p2) {
        int c = 0;
        for (int q1 = 0; q1 < NP; ++q1)
            for (int q2 = 0; q2 < NP; ++q2)
                if (linked(q1, q2)) {
                    if (q1 == p1 && q2 == p2) return c;
                    ++c;
                }
        return -1;
    }
    // pairs of class c, in pair order
    static constexpr int class_size(int c) {
        int n = 0;
        for (int p = 0; p < NP; ++p)
            if (cls(p) == c) ++n;
        return n;
    }
    static constexpr int class_member(int c, int r) {
        int n = 0;
        for (int p = 0; p < NP; ++p)
            if (cls(p) == c) {
                if (n == r) return p;
                ++n;
            }
        return -1;
    }
    static constexpr int max_class_size() {
        int m = 0;
        for (int c = 0; c < M; ++c)
            if (class_size(c) > m) m = class_size(c);
        return m;
    }
};

// Runtime (host) versions of the same enumeration.
inline int n_pairs(int M) { return M * (M + 1) / 2; }

struct SecInfo {
    int N, P, dim, pad;
    long long off;
};

struct Tile {
    int sec, row0, nrows, pad;
};

// Epilogue of the fused stage kernel.  With h = (H x)(row) and k = ks * h:
//   APPLY : out      = h
//   FIRST : acc      = base + a k ;  ynext = c0 base + b k
//   MID   : acc      = acc  + a k ;  ynext = c0 base + b k
//   LAST  : baseout  = acc  + a k
enum StageMode { kApply = 0, kFirst = 1, kMid = 2, kLast = 3 };

struct StageArgs {
    const double* x;      // gathered vector, complex interleaved
    double* out;
    const double* base;
    double* acc;
    double* ynext;
    double* baseout;
    double ks_re, ks_im;
    double a, c0, b;
    int mode;
    const int* T;         // rank table (ints)
    int Tn;               // number of ints
    int Rdim;             // Nmax + 5
    const double* coef;   // omega[M] | Wd[NP] | W[NC]
    int ncoef;
    const double* sqrt_tab;  // sqrt(0..Nmax+2)
    int nsqrt;
    const Tile* tiles;
    int ntiles;
    const SecInfo* secs;
    int xcd_order;
    unsigned* queue;      // xcd_order 3: one tile counter per XCD, zero at launch; null: static walk
};

// Moments / one-body kernels.
struct MomArgs {
    const double* psi;
    int nrhs, rhs;
    const int* T;
    int Tn, Rdim;
    const double* sqrt_tab;
    int nsqrt;
    const Tile* tiles;
    int ntiles;
    const SecInfo* secs;
    const int* secmap;  // [(N) * M + P] -> sector id or -1, N in [0, Nmax]
    int Nmax;
    double* partial;    // [group][grid][kMomOut] complex
    int xcd_order;
    const unsigned char* occ;  // occupation records
};
constexpr int momentsOut(int M) { return 2 * M + 1; }
// LDS layout of the table-staging kernels: rank table (ints, padded to an even
// count), then the sqrt table (doubles), then reduction space.
FH_HD constexpr int lds_sqrt_offset(int Tn) { return (Tn + 1) & ~1; }
constexpr int kMomOutMax = 2 * kMaxM + 1;

// One-body source  g(n) = c0 x(n) + cN N(n) x(n) + sum_i u_i (a_i x)(n)
//                        + sum_i v_i (a_i^+ x)(n) + sum_ij h_ij (a_i^+ a_j x)(n)
struct OneBodyArgs {
    const double* psi;
    double* out;
    int nrhs, rhs;
    const int* T;
    int Tn, Rdim;
    const double* sqrt_tab;
    int nsqrt;
    const Tile* tiles;
    int ntiles;
    const SecInfo* secs;
    const int* secmap;
    int Nmax;
    const double* cf;   // c0(2), cN(2), u[M](2), v[M](2), h[M*M](2)
};

// Occupation records: the occupations of every state of a basis, one byte per
// mode, padded to occ_stride(M) bytes, at the state's global index.
constexpr FH_HD int occ_stride(int M) { return M <= 8 ? 8 : 16; }
struct OccArgs {
    const int* T;
    int Tn, Rdim;
    const Tile* tiles;
    int ntiles;
    const SecInfo* secs;
    unsigned char* occ;
};

// Quartic correlators  G[c][(p1,p2)] = sum_q sum_n conj(uscale_q u_q(n)) <n|a_i^+ a_j^+ a_k a_l|n'> y_q(n')
// for pairs p1 = {i,j}, p2 = {k,l} of class c (p1 == p2 included), summed over
// kCorrPairs vector pairs (u_q, y_q) at once (the four stages of an adjoint step).
// Only Im G is computed (the real parts are written as 0): with V real the
// gradients need Im G alone.
constexpr int kCorrPairs = 4;
// pairs handled by one correlator launch (registers: M >= 9 has classes of 6 pairs)
constexpr FH_HD int corr_pairs_per_launch(int M) { return M >= 9 ? 2 : kCorrPairs; }
struct CorrArgs {
    const unsigned char* occ;  // occupation records
    const double* u[kCorrPairs];
    const double* y[kCorrPairs];
    double uscale[kCorrPairs];
    int nrhs, rhs;
    const int* T;
    int Tn, Rdim;
    const double* sqrt_tab;
    int nsqrt;
    const Tile* tiles;
    int ntiles;
    const SecInfo* secs;
    double* partial;    // [class][grid][kCorrOutMax] complex
    int xcd_order;
    unsigned* queue;    // xcd_order 3: tile counters [class][XCD], zero at launch
};
constexpr int kCorrOutMax = 36;  // (max class size)^2 for M <= 10

// Classical (mean-field) trajectories, one per thread.
struct ClassicalArgs {
    double* alpha;        // [ntraj][M] complex, in/out
    double* out;          // [nout][ntraj][M] complex, or nullptr
    const double* omega;  // [M]
    const double* U;      // [M][M][M]: U[p][j][k] = (Lambda/2)(V_pjkl + V_jpkl), l = p + j - k mod M
    double dt;
    long long nsteps, every;
    int ntraj;
};

// Initial states.
struct InitArgs {
    double* psi;
    int nrhs;
    const int* T;
    int Tn, Rdim;
    const Tile* tiles;
    int ntiles;
    const SecInfo* secs;
    const double* tab;  // [rhs][M][Nmax+1] complex: per-mode factors
    int Nmax;
};

// Coherent-state vector-Jacobian product: per rhs, sums
//   S0 = sum conj(g) psi0,  S_k = sum conj(g) psi0 with factor k replaced by tabd.
struct VjpArgs {
    const double* g;
    int nrhs, rhs;
    const int* T;
    int Tn, Rdim;
    const Tile* tiles;
    int ntiles;
    const SecInfo* secs;
    const double* tab;   // [M][Nmax+1] complex factors of psi0 (this rhs)
    const double* tabd;  // [M][Nmax+1] complex factors n a^(n-1)/sqrt(n!) e^{-|a|^2/2}
    int Nmax;
    double* partial;     // [grid][kMaxM+1] complex
};

struct RankArgs {
    const uint8_t* occ;
    const int64_t* idx_in;
    int64_t* idx;
    uint8_t* occ_out;
    long long count;
    int N, P, dim;
    const int* T;
    int Tn, Rdim;
};

}  // namespace fh

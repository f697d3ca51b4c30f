// fh_host.hpp -- host-side handle definitions and helpers (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/fockhip.h"
#include "fh_common.hpp"
#include "fh_launch.hpp"

struct fh_model {
    int M = 0, pmod = 0;
    std::vector<double> omega;   // [M]
    std::vector<double> V;       // [M^4]
    double Lambda = 0.0;
    std::vector<double> coef;    // omega[M] | Wd[NP] | W[NC] | U[M^3] (classical field)
    size_t ucoef_off = 0;        // offset of U in coef
    double* d_coef = nullptr;
    int device = 0;
};

struct fh_basis {
    int M = 0, pmod = 0, nsec = 0, Nmax = 0;
    std::vector<int> N, P;
    std::vector<int64_t> dim, off;
    int64_t total = 0;
    int Rdim = 0, Tn = 0;
    std::vector<int> T;            // rank table, device layout
    std::vector<double> sqrt_tab;  // sqrt(0 .. Nmax + 2)
    std::vector<int64_t> D;        // host counting table D[m][R][Q], R in [0, Nmax+2]
    std::vector<fh::SecInfo> secs;
    std::vector<fh::Tile> tiles;
    std::vector<int> tile_begin;   // [nsec + 1]
    std::vector<int> secmap;       // [(Nmax+1) * M]
    // device copies
    int* d_T = nullptr;
    double* d_sqrt = nullptr;
    fh::SecInfo* d_secs = nullptr;
    fh::Tile* d_tiles = nullptr;
    int* d_secmap = nullptr;
    unsigned* d_queue = nullptr;   // xcd_order 3: tile counters ([class][XCD] for the correlators)
    double* d_partial = nullptr;   // reduction partials
    size_t partial_doubles = 0;
    double* d_small = nullptr;     // reduced values, coefficient tables, ...
    size_t small_doubles = 0;
    unsigned char* d_occ = nullptr;  // occupation record of every state (occ_stride(M) bytes)
    int device = 0;
    int num_cu = 0;
    int grid_cap = 0;              // max persistent workgroups
    int blocks_per_cu = 0;         // 0 = occupancy limit
    int xcd_order = 3;             // fh_basis_set_launch; 3 = per-XCD tile queues over interleaved chunks
    int tile_order = 0;            // fh_basis_set_tile_order
    int prefix_modes = 0;
    const fh::KernelSet* ks = nullptr;

    int64_t D_at(int m, int R, int Q) const {
        if (R < 0) return 0;
        return D[((size_t)m * (Nmax + 3) + R) * pmod + Q];
    }
};

namespace fh {
constexpr size_t kQueueBytes = 8 * kMaxM * sizeof(unsigned);  // tile counters of XCD order 3
void set_error(const std::string& msg);
fh_status hip_fail(hipError_t e, const char* what);
size_t lds_bytes(const fh_basis* b, int extra_doubles);
int persistent_grid(const fh_basis* b, const void* fn, size_t lds, int ntiles);
bool use_queue(const fh_basis* b, long long units, int grid);
int moments_grid(const fh_basis* b, size_t* lds);
fh_status moments_core(const fh_basis* b, int nrhs, int rhs, const double* psi, double* rec, hipStream_t s,
                       int groups, double* partial, double* reduced, double* v);
}  // namespace fh

#define FH_HIP(call)                                       \
    do {                                                   \
        hipError_t _e = (call);                            \
        if (_e != hipSuccess) return fh::hip_fail(_e, #call); \
    } while (0)

#define FH_REQUIRE(cond, code, msg)   \
    do {                              \
        if (!(cond)) {                \
            fh::set_error(msg);       \
            return (code);            \
        }                             \
    } while (0)

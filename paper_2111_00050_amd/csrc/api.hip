// api.hip -- the C ABI of fockhip.h: handles, tables, launches and host loops.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstdio>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <utility>
#include <vector>

#include "fh_host.hpp"

namespace fh {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

fh_status hip_fail(hipError_t e, const char* what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return FH_EHIP;
}

size_t lds_bytes(const fh_basis* b, int extra_doubles) {
    return sizeof(int) * (size_t)lds_sqrt_offset(b->Tn) + sizeof(double) * (b->sqrt_tab.size() + extra_doubles);
}

static std::mutex g_occ_mu;
static std::map<std::pair<const void*, size_t>, int> g_occ;

int persistent_grid(const fh_basis* b, const void* fn, size_t lds, int ntiles) {
    int per_cu = 0;
    {
        std::lock_guard<std::mutex> lk(g_occ_mu);
        auto key = std::make_pair(fn, lds);
        auto it = g_occ.find(key);
        if (it != g_occ.end()) {
            per_cu = it->second;
        } else {
            int nb = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, kTileRows, lds) != hipSuccess || nb < 1) nb = 1;
            g_occ[key] = nb;
            per_cu = nb;
        }
    }
    if (b->blocks_per_cu > 0) per_cu = std::min(per_cu, b->blocks_per_cu);
    long long G = (long long)b->num_cu * per_cu;
    if (G > b->grid_cap) G = b->grid_cap;
    if (G > ntiles) G = ntiles;
    if (G < 1) G = 1;
    return (int)G;
}

// Walk order 3 takes the units from per-XCD counters only where every
// workgroup takes many of them: a short launch (a few units per workgroup)
// walks statically (as order 1), without the counter fill and the
// per-unit barriers and atomics, which there cost more than the locality gains.
constexpr int kQueueMinUnitsPerBlock = 16;
bool use_queue(const fh_basis* b, long long units, int grid) {
    return b->xcd_order == 3 && (grid & 7) == 0 && units >= (long long)kQueueMinUnitsPerBlock * grid;
}

}  // namespace fh

using namespace fh;

namespace {

int posmod(long long a, int m) {
    long long r = a % m;
    return (int)(r < 0 ? r + m : r);
}

struct Guard {  // catches C++ exceptions at the ABI boundary
    template <class F>
    static fh_status run(F&& f) {
        try {
            return f();
        } catch (const std::bad_alloc&) {
            set_error("host allocation failed");
            return FH_ENOMEM;
        } catch (const std::exception& e) {
            set_error(std::string("internal error: ") + e.what());
            return FH_EINVAL;
        } catch (...) {
            set_error("internal error");
            return FH_EINVAL;
        }
    }
};

// Pair orderings: {(i,j)} or {(i,j),(j,i)}.
void orderings(int i, int j, int out[2][2], int* n) {
    out[0][0] = i;
    out[0][1] = j;
    *n = 1;
    if (i != j) {
        out[1][0] = j;
        out[1][1] = i;
        *n = 2;
    }
}

// Coefficient table omega[M] | Wd[NP] | W[NC] (enumeration of fh_common.hpp).
void build_coef(fh_model* m) {
    const int M = m->M, NP = n_pairs(M);
    std::vector<int> pi(NP), pj(NP);
    int c = 0;
    for (int a = 0; a < M; ++a)
        for (int b = a; b < M; ++b) {
            pi[c] = a;
            pj[c] = b;
            ++c;
        }
    auto Vat = [&](int i, int j, int k, int l) { return m->V[(((size_t)i * M + j) * M + k) * M + l]; };
    auto pairsum = [&](int p1, int p2) {
        int o1[2][2], o2[2][2], n1, n2;
        orderings(pi[p1], pj[p1], o1, &n1);
        orderings(pi[p2], pj[p2], o2, &n2);
        double s = 0.0;
        for (int x = 0; x < n1; ++x)
            for (int y = 0; y < n2; ++y) s += Vat(o1[x][0], o1[x][1], o2[y][0], o2[y][1]);
        return 0.5 * m->Lambda * s;
    };
    m->coef.assign(m->omega.begin(), m->omega.end());
    for (int p = 0; p < NP; ++p) m->coef.push_back(pairsum(p, p));
    auto cls = [&](int p) { return (pi[p] + pj[p]) % M; };
    for (int p1 = 0; p1 < NP; ++p1)
        for (int p2 = 0; p2 < NP; ++p2)
            if (p1 != p2 && cls(p1) == cls(p2)) m->coef.push_back(pairsum(p1, p2));
    // classical field: U[p][j][k] = (Lambda/2)(V_pjkl + V_jpkl), l = p + j - k mod M
    m->ucoef_off = m->coef.size();
    for (int p = 0; p < M; ++p)
        for (int j = 0; j < M; ++j)
            for (int k = 0; k < M; ++k) {
                const int l = posmod(p + j - k, M);
                m->coef.push_back(0.5 * m->Lambda * (Vat(p, j, k, l) + Vat(j, p, k, l)));
            }
}

fh_status model_upload(fh_model* m) {
    FH_HIP(hipGetDevice(&m->device));
    FH_HIP(hipMalloc(&m->d_coef, sizeof(double) * m->coef.size()));
    FH_HIP(hipMemcpy(m->d_coef, m->coef.data(), sizeof(double) * m->coef.size(), hipMemcpyHostToDevice));
    return FH_OK;
}

fh_status make_model(int M, int pmod, const double* omega, double Lambda, const double* V, fh_model** out) {
    FH_REQUIRE(out != nullptr, FH_EINVAL, "fh_model_create: out is NULL");
    *out = nullptr;
    FH_REQUIRE(M >= 1 && M <= kMaxM, FH_EUNSUPPORTED, "fh_model_create: M must be in [1, 10]");
    FH_REQUIRE(pmod == M, FH_EUNSUPPORTED, "fh_model_create: the GPU path supports pmod == M only");
    FH_REQUIRE(omega != nullptr && V != nullptr, FH_EINVAL, "fh_model_create: omega or V is NULL");
    FH_REQUIRE(std::isfinite(Lambda), FH_EINVAL, "fh_model_create: Lambda is not finite");
    const size_t m4 = (size_t)M * M * M * M;
    for (int j = 0; j < M; ++j) FH_REQUIRE(std::isfinite(omega[j]), FH_EINVAL, "fh_model_create: omega not finite");
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < M; ++j)
            for (int k = 0; k < M; ++k)
                for (int l = 0; l < M; ++l) {
                    const double v = V[(((size_t)i * M + j) * M + k) * M + l];
                    FH_REQUIRE(std::isfinite(v), FH_EINVAL, "fh_model_create: V not finite");
                    if (v != 0.0 && posmod(i + j - k - l, pmod) != 0) {
                        set_error("fh_model_create: V[" + std::to_string(i) + "][" + std::to_string(j) + "][" +
                                  std::to_string(k) + "][" + std::to_string(l) +
                                  "] is nonzero but does not conserve momentum");
                        return FH_EINVAL;
                    }
                }
    auto* m = new fh_model();
    m->M = M;
    m->pmod = pmod;
    m->omega.assign(omega, omega + M);
    m->V.assign(V, V + m4);
    m->Lambda = Lambda;
    build_coef(m);
    fh_status st = model_upload(m);
    if (st != FH_OK) {
        if (m->d_coef) (void)hipFree(m->d_coef);
        delete m;
        return st;
    }
    *out = m;
    return FH_OK;
}

// ---------------------------------------------------------------- basis --
constexpr int64_t kCap = (int64_t)1 << 62;

fh_status build_tables(fh_basis* b) {
    const int M = b->M, p = b->pmod, W = b->Nmax + 3;
    // D[m][R][Q] for m = M..0, R = 0..Nmax+2 (saturating at 2^62)
    b->D.assign((size_t)(M + 1) * W * p, 0);
    b->D[((size_t)M * W + 0) * p + 0] = 1;
    for (int m = M - 1; m >= 0; --m)
        for (int R = 0; R < W; ++R)
            for (int Q = 0; Q < p; ++Q) {
                int64_t s = 0;
                for (int v = 0; v <= R; ++v) {
                    s += b->D[((size_t)(m + 1) * W + (R - v)) * p + posmod((long long)Q - (long long)m * v, p)];
                    if (s > kCap) s = kCap;
                }
                b->D[((size_t)m * W + R) * p + Q] = s;
            }
    // T_s(R, Q) = D_{s-1}(R - 1, Q - (s - 1)), s = 1..M-1, R = -2..Nmax+2, Q stored twice.
    b->Rdim = b->Nmax + 5;
    const int P2 = 2 * p;
    b->Tn = std::max(1, (M - 1) * b->Rdim * P2);
    b->T.assign(b->Tn, 0);
    for (int s = 1; s < M; ++s)
        for (int R = -kRBias; R <= b->Nmax + 2; ++R)
            for (int q = 0; q < P2; ++q) {
                int64_t v = 0;
                if (R >= 1) v = b->D_at(s - 1, R - 1, posmod(q - (s - 1), p));
                if (v > INT32_MAX) {
                    // Only reachable from configurations with more than Nmax bosons
                    // (never formed by a valid move); a sector that needs it is
                    // rejected by the dimension check below.
                    if (R - 1 <= b->Nmax) {
                        set_error("fh_basis_create: counting table entry exceeds 2^31-1");
                        return FH_EOVERFLOW;
                    }
                    v = INT32_MAX;
                }
                b->T[(size_t)(s - 1) * b->Rdim * P2 + (size_t)(R + kRBias) * P2 + q] = (int)v;
            }
    b->sqrt_tab.resize(b->Nmax + 3);
    for (int x = 0; x < (int)b->sqrt_tab.size(); ++x) b->sqrt_tab[x] = std::sqrt((double)x);
    return FH_OK;
}

void basis_free(fh_basis* b) {
    if (!b) return;
    (void)hipFree(b->d_T);
    (void)hipFree(b->d_sqrt);
    (void)hipFree(b->d_secs);
    (void)hipFree(b->d_tiles);
    (void)hipFree(b->d_secmap);
    (void)hipFree(b->d_queue);
    (void)hipFree(b->d_partial);
    (void)hipFree(b->d_small);
    (void)hipFree(b->d_occ);
    delete b;
}

fh_status make_basis(int M, int pmod, int nsec, const int32_t* N, const int32_t* P, fh_basis** out) {
    FH_REQUIRE(out != nullptr, FH_EINVAL, "fh_basis_create: out is NULL");
    *out = nullptr;
    FH_REQUIRE(M >= 1 && M <= kMaxM, FH_EUNSUPPORTED, "fh_basis_create: M must be in [1, 10]");
    FH_REQUIRE(pmod == M, FH_EUNSUPPORTED, "fh_basis_create: the GPU path supports pmod == M only");
    FH_REQUIRE(nsec >= 1, FH_EINVAL, "fh_basis_create: need at least one sector");
    FH_REQUIRE(N != nullptr && P != nullptr, FH_EINVAL, "fh_basis_create: N or P is NULL");
    std::set<std::pair<int, int>> seen;
    int Nmax = 0;
    for (int s = 0; s < nsec; ++s) {
        FH_REQUIRE(N[s] >= 0 && N[s] <= 253, FH_EINVAL, "fh_basis_create: N must be in [0, 253]");
        FH_REQUIRE(P[s] >= 0 && P[s] < pmod, FH_EINVAL, "fh_basis_create: P must be in [0, pmod)");
        FH_REQUIRE(seen.insert({N[s], P[s]}).second, FH_EINVAL, "fh_basis_create: duplicate sector");
        Nmax = std::max(Nmax, (int)N[s]);
    }
    auto* b = new fh_basis();
    b->M = M;
    b->pmod = pmod;
    b->nsec = nsec;
    b->Nmax = Nmax;
    b->N.assign(N, N + nsec);
    b->P.assign(P, P + nsec);
    b->ks = kernel_set(M);
    fh_status st = build_tables(b);
    if (st != FH_OK) {
        delete b;
        return st;
    }
    // LDS budget: rank table + sqrt table + reduction space must fit comfortably.
    if (lds_bytes(b, 4 * 2 * kCorrOutMax) > 96 * 1024) {
        delete b;
        set_error("fh_basis_create: rank table too large for LDS (reduce Nmax or M)");
        return FH_EUNSUPPORTED;
    }
    b->dim.resize(nsec);
    b->off.resize(nsec + 1);
    int64_t off = 0;
    for (int s = 0; s < nsec; ++s) {
        const int64_t d = b->D_at(0, N[s], P[s]);
        if (d >= ((int64_t)1 << 28)) {
            // Single-rhs gathers use 32-bit byte offsets inside a sector.
            delete b;
            set_error("fh_basis_create: a sector has 2^28 or more states (limit of this build)");
            return FH_EOVERFLOW;
        }
        b->dim[s] = d;
        b->off[s] = off;
        off += d;
    }
    b->off[nsec] = off;
    b->total = off;
    b->secs.resize(nsec);
    b->tile_begin.resize(nsec + 1);
    for (int s = 0; s < nsec; ++s) {
        b->secs[s] = SecInfo{N[s], P[s], (int)b->dim[s], 0, (long long)b->off[s]};
        b->tile_begin[s] = (int)b->tiles.size();
        for (int64_t r = 0; r < b->dim[s]; r += kTileRows)
            b->tiles.push_back(Tile{s, (int)r, (int)std::min<int64_t>(kTileRows, b->dim[s] - r), 0});
    }
    b->tile_begin[nsec] = (int)b->tiles.size();
    // the stage kernel walks up to 4 passes per tile in int arithmetic
    if (b->tiles.size() > (size_t)INT32_MAX / 4) {
        delete b;
        set_error("fh_basis_create: too many tiles");
        return FH_EOVERFLOW;
    }
    b->secmap.assign((size_t)(Nmax + 1) * M, -1);
    for (int s = 0; s < nsec; ++s) b->secmap[(size_t)N[s] * M + P[s]] = s;

    auto fail = [&](hipError_t e, const char* what) {
        basis_free(b);
        return hip_fail(e, what);
    };
    hipError_t e;
    if ((e = hipGetDevice(&b->device)) != hipSuccess) return fail(e, "hipGetDevice");
    if ((e = hipDeviceGetAttribute(&b->num_cu, hipDeviceAttributeMultiprocessorCount, b->device)) != hipSuccess)
        return fail(e, "hipDeviceGetAttribute");
    b->grid_cap = b->num_cu * 8;
    b->partial_doubles = (size_t)std::max(M + 1, kMaxM) * b->grid_cap * 2 * std::max(kMomOutMax, kCorrOutMax);
    b->small_doubles = (size_t)16 * M * (Nmax + 3) * 2 * 2 + 4 * (size_t)kMaxM * 2 * kCorrOutMax + 65536;
    const size_t ntile = std::max<size_t>(1, b->tiles.size());
    if ((e = hipMalloc(&b->d_T, sizeof(int) * b->T.size())) != hipSuccess) return fail(e, "hipMalloc");
    if ((e = hipMalloc(&b->d_sqrt, sizeof(double) * b->sqrt_tab.size())) != hipSuccess) return fail(e, "hipMalloc");
    if ((e = hipMalloc(&b->d_secs, sizeof(SecInfo) * nsec)) != hipSuccess) return fail(e, "hipMalloc");
    if ((e = hipMalloc(&b->d_tiles, sizeof(Tile) * ntile)) != hipSuccess) return fail(e, "hipMalloc");
    if ((e = hipMalloc(&b->d_secmap, sizeof(int) * b->secmap.size())) != hipSuccess) return fail(e, "hipMalloc");
    if ((e = hipMalloc(&b->d_partial, sizeof(double) * b->partial_doubles)) != hipSuccess) return fail(e, "hipMalloc");
    if ((e = hipMalloc(&b->d_queue, kQueueBytes)) != hipSuccess) return fail(e, "hipMalloc");
    if ((e = hipMalloc(&b->d_small, sizeof(double) * b->small_doubles)) != hipSuccess) return fail(e, "hipMalloc");
    if ((e = hipMemcpy(b->d_T, b->T.data(), sizeof(int) * b->T.size(), hipMemcpyHostToDevice)) != hipSuccess)
        return fail(e, "hipMemcpy");
    if ((e = hipMemcpy(b->d_sqrt, b->sqrt_tab.data(), sizeof(double) * b->sqrt_tab.size(), hipMemcpyHostToDevice)) !=
        hipSuccess)
        return fail(e, "hipMemcpy");
    if ((e = hipMemcpy(b->d_secs, b->secs.data(), sizeof(SecInfo) * nsec, hipMemcpyHostToDevice)) != hipSuccess)
        return fail(e, "hipMemcpy");
    if (!b->tiles.empty() &&
        (e = hipMemcpy(b->d_tiles, b->tiles.data(), sizeof(Tile) * b->tiles.size(), hipMemcpyHostToDevice)) !=
            hipSuccess)
        return fail(e, "hipMemcpy");
    if ((e = hipMemcpy(b->d_secmap, b->secmap.data(), sizeof(int) * b->secmap.size(), hipMemcpyHostToDevice)) !=
        hipSuccess)
        return fail(e, "hipMemcpy");
    // occupation records (occ_stride(M) bytes per state), filled once here
    if ((e = hipMalloc(&b->d_occ, (size_t)occ_stride(M) * std::max<int64_t>(1, b->total))) != hipSuccess)
        return fail(e, "hipMalloc");
    if (!b->tiles.empty()) {
        OccArgs oa{};
        oa.T = b->d_T;
        oa.Tn = b->Tn;
        oa.Rdim = b->Rdim;
        oa.tiles = b->d_tiles;
        oa.ntiles = (int)b->tiles.size();
        oa.secs = b->d_secs;
        oa.occ = b->d_occ;
        const size_t lds = sizeof(int) * b->Tn;
        b->ks->occ_table(oa, std::min(oa.ntiles, 4 * b->num_cu), lds, nullptr);
        if ((e = hipGetLastError()) != hipSuccess) return fail(e, "occ_table_kernel");
        if ((e = hipStreamSynchronize(nullptr)) != hipSuccess) return fail(e, "hipStreamSynchronize");
    }
    *out = b;
    return FH_OK;
}

// Lexicographic rank on the host: sum over modes of the number of sector
// states with a smaller entry at the first differing mode.
int64_t host_rank(const fh_basis* b, int sec, const uint8_t* occ) {
    const int M = b->M, p = b->pmod;
    int R = b->N[sec], Q = b->P[sec];
    int64_t r = 0;
    for (int m = 0; m < M; ++m) {
        for (int v = 0; v < occ[m]; ++v) r += b->D_at(m + 1, R - v, posmod((long long)Q - (long long)m * v, p));
        R -= occ[m];
        Q = posmod((long long)Q - (long long)m * occ[m], p);
    }
    return r;
}

// Inverse of host_rank: the occupation vector at rank r of sector sec.
void host_unrank(const fh_basis* b, int sec, int64_t r, int* occ) {
    const int M = b->M, p = b->pmod;
    int R = b->N[sec], Q = b->P[sec];
    for (int m = 0; m < M - 1; ++m) {
        int v = 0;
        while (v < R) {
            const int64_t cnt = b->D_at(m + 1, R - v, posmod((long long)Q - (long long)m * v, p));
            if (r < cnt) break;
            r -= cnt;
            ++v;
        }
        occ[m] = v;
        R -= v;
        Q = posmod((long long)Q - (long long)m * v, p);
    }
    occ[M - 1] = R;
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

bool check_model_basis(const fh_model* m, const fh_basis* b) {
    if (!m || !b) {
        set_error("model or basis is NULL");
        return false;
    }
    if (m->M != b->M || m->pmod != b->pmod) {
        set_error("model and basis disagree on M or pmod");
        return false;
    }
    return true;
}

bool bad_nrhs(int nrhs) { return nrhs_slot(nrhs) < 0; }

StageArgs stage_base(const fh_model* m, const fh_basis* b) {
    StageArgs a{};
    a.T = b->d_T;
    a.Tn = b->Tn;
    a.Rdim = b->Rdim;
    a.coef = m->d_coef;
    a.ncoef = (int)m->coef.size();
    a.sqrt_tab = b->d_sqrt;
    a.nsqrt = (int)b->sqrt_tab.size();
    a.secs = b->d_secs;
    a.xcd_order = b->xcd_order;
    a.queue = nullptr;  // chosen per launch
    return a;
}

struct StageTimer {
    bool on = false;
    std::vector<hipEvent_t> ev;  // pairs
    size_t used = 0;
    double ms = 0.0;
    int64_t launches = 0;
    hipStream_t s = nullptr;
    fh_status init(bool enable, hipStream_t st) {
        on = enable;
        s = st;
        if (!on) return FH_OK;
        ev.resize(512);
        for (auto& e : ev) FH_HIP(hipEventCreate(&e));
        return FH_OK;
    }
    fh_status flush() {
        if (!on || used == 0) return FH_OK;
        FH_HIP(hipEventSynchronize(ev[used - 1]));
        for (size_t q = 0; q < used; q += 2) {
            float t = 0.f;
            FH_HIP(hipEventElapsedTime(&t, ev[q], ev[q + 1]));
            ms += t;
        }
        used = 0;
        return FH_OK;
    }
    fh_status begin() {
        if (!on) return FH_OK;
        if (used + 2 > ev.size()) {
            fh_status st = flush();
            if (st != FH_OK) return st;
        }
        FH_HIP(hipEventRecord(ev[used], s));
        return FH_OK;
    }
    fh_status end() {
        if (!on) return FH_OK;
        FH_HIP(hipEventRecord(ev[used + 1], s));
        used += 2;
        ++launches;
        return FH_OK;
    }
    ~StageTimer() {
        for (auto& e : ev) (void)hipEventDestroy(e);
    }
};

// One stage over all sectors (persistent launch) or one launch per sector.
// With 16 right-hand sides at M >= 9 (one wave per SIMD) the fused RK4
// epilogue's once-per-row loads wait at the end of every row; there a stage
// is an H y pass into its destination buffer followed by a streaming update
// pass (measured at M = 10: 1100 -> 1005 ms per stage; with one column the
// split is 3 % slower, so one column keeps the fused epilogue).
inline bool split_epilogue(int M, int nrhs) { return M >= 9 && nrhs >= 16; }

fh_status launch_stage(const fh_basis* b, int nrhs, StageArgs a, int flags, hipStream_t s, StageTimer* tm) {
    const int slot = nrhs_slot(nrhs);
    const int mode = a.mode;
    const bool split = mode != kApply && split_epilogue(b->M, nrhs);
    if (split) {
        // H y goes to the buffer the update writes (next, or baseout for the
        // last stage); neither is read by the stage kernel itself.
        a.out = mode == kLast ? a.baseout : a.ynext;
        a.mode = kApply;
    }
    const void* fn = b->ks->stage_fn[slot];
    const size_t lds = lds_bytes(b, 0);
    const int G = stage_lanes_per_row(nrhs);  // workgroup passes per tile
    if (tm) {
        fh_status st = tm->begin();
        if (st != FH_OK) return st;
    }
    if (flags & FH_PER_SECTOR) {
        for (int sec = 0; sec < b->nsec; ++sec) {
            const int nt = b->tile_begin[sec + 1] - b->tile_begin[sec];
            if (nt == 0) continue;
            a.tiles = b->d_tiles + b->tile_begin[sec];
            a.ntiles = nt;
            a.queue = nullptr;  // per-sector launches walk their tiles statically (order 3 as order 1)
            b->ks->stage[slot](a, persistent_grid(b, fn, lds, nt * G), lds, s);
        }
    } else {
        const int nt = (int)b->tiles.size();
        if (nt > 0) {
            a.tiles = b->d_tiles;
            a.ntiles = nt;
            const int grid = persistent_grid(b, fn, lds, nt * G);
            a.queue = b->M >= kStageCounterMinM && use_queue(b, nt * G, grid) ? b->d_queue : nullptr;
            if (a.queue) {
                // the eight XCD counters start at zero (a fill kernel: also valid under graph capture)
                launch_fill(reinterpret_cast<double*>(b->d_queue), 4, 0.0, s);
                FH_HIP(hipGetLastError());
            }
            b->ks->stage[slot](a, grid, lds, s);
        }
    }
    FH_HIP(hipGetLastError());
    if (split) {
        launch_rk4_update(a.out, a.base, a.acc, a.ynext, a.baseout, (long long)b->total * nrhs, mode, a.ks_re, a.ks_im,
                          a.a, a.c0, a.b, s);
        FH_HIP(hipGetLastError());
    }
    if (tm) return tm->end();
    return FH_OK;
}

}  // namespace

namespace fh {
// Workgroups of the moments launch for this basis and its dynamic LDS bytes.
int moments_grid(const fh_basis* b, size_t* lds) {
    const int NO = momentsOut(b->M);
    *lds = lds_bytes(b, 4 * 2 * NO);
    const int nt = (int)b->tiles.size();
    return nt > 0 ? persistent_grid(b, b->ks->moments_fn, *lds, nt) : 0;
}

// Moments of one rhs into host doubles rec = [norm2, a(2M), M(2M^2), A(2M^2)].
// Scratch: partial holds groups * G * 2 * kMomOutMax doubles (G = moments_grid),
// reduced groups * 2 * momentsOut(M) doubles (device); v is host staging of
// groups * 2 * momentsOut(M) doubles.  Every scratch word read is written first.
fh_status moments_core(const fh_basis* b, int nrhs, int rhs, const double* psi, double* rec, hipStream_t s,
                       int groups, double* partial, double* reduced, double* v) {
    const int M = b->M, NO = momentsOut(M);
    const int nt = (int)b->tiles.size();
    size_t lds = 0;
    const int G = moments_grid(b, &lds);
    MomArgs a{};
    a.psi = psi;
    a.nrhs = nrhs;
    a.rhs = rhs;
    a.T = b->d_T;
    a.Tn = b->Tn;
    a.Rdim = b->Rdim;
    a.sqrt_tab = b->d_sqrt;
    a.nsqrt = (int)b->sqrt_tab.size();
    a.tiles = b->d_tiles;
    a.ntiles = nt;
    a.secs = b->d_secs;
    a.secmap = b->d_secmap;
    a.Nmax = b->Nmax;
    a.partial = partial;
    a.xcd_order = b->xcd_order;
    a.occ = b->d_occ;
    const size_t nv = (size_t)groups * 2 * NO;
    std::fill(v, v + nv, 0.0);
    if (nt > 0) {
        b->ks->moments(a, G, groups, lds, s);
        FH_HIP(hipGetLastError());
        launch_reduce_partials(partial, groups, G, 2 * kMomOutMax, 2 * NO, reduced, 0, s);
        FH_HIP(hipGetLastError());
        FH_HIP(hipMemcpyAsync(v, reduced, sizeof(double) * nv, hipMemcpyDeviceToHost, s));
        FH_HIP(hipStreamSynchronize(s));
    }
    const size_t need = FH_MOMENT_DOUBLES(M);
    std::fill(rec, rec + need, 0.0);
    double* ra = rec + 1;
    double* rM = rec + 1 + 2 * M;
    double* rA = rec + 1 + 2 * M + 2 * M * M;
    auto g = [&](int grp, int slot, int c) { return v[(size_t)grp * 2 * NO + 2 * slot + c]; };
    rec[0] = g(0, 0, 0);
    for (int i = 0; i < M; ++i) {
        ra[2 * i] = g(0, 1 + i, 0);
        ra[2 * i + 1] = g(0, 1 + i, 1);
        rM[2 * (i * M + i)] = g(0, 1 + M + i, 0);
    }
    if (groups > 1) {
        for (int i = 0; i < M; ++i) {
            for (int j = 0; j < M; ++j)
                if (j != i) {
                    rM[2 * (i * M + j)] = g(1 + i, j, 0);
                    rM[2 * (i * M + j) + 1] = g(1 + i, j, 1);
                }
            for (int l = i; l < M; ++l) {
                const double re = g(1 + i, M + l, 0), im = g(1 + i, M + l, 1);
                rA[2 * (i * M + l)] = re;
                rA[2 * (i * M + l) + 1] = im;
                rA[2 * (l * M + i)] = re;
                rA[2 * (l * M + i) + 1] = im;
            }
        }
    }
    return FH_OK;
}
}  // namespace fh

namespace {

// Moments of one rhs with the basis's own scratch.
fh_status run_moments(const fh_basis* b, int nrhs, int rhs, const double* psi, double* rec, hipStream_t s,
                      int groups) {
    std::vector<double> v((size_t)groups * 2 * momentsOut(b->M));
    return moments_core(b, nrhs, rhs, psi, rec, s, groups, b->d_partial, b->d_small, v.data());
}

fh_status init_product(const fh_basis* b, int nrhs, const std::vector<double>& tab, double* psi, hipStream_t s) {
    FH_REQUIRE(tab.size() <= b->small_doubles, FH_EUNSUPPORTED, "initial-state table too large");
    FH_HIP(hipMemcpyAsync(b->d_small, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice, s));
    InitArgs a{};
    a.psi = psi;
    a.nrhs = nrhs;
    a.T = b->d_T;
    a.Tn = b->Tn;
    a.Rdim = b->Rdim;
    a.tiles = b->d_tiles;
    a.ntiles = (int)b->tiles.size();
    a.secs = b->d_secs;
    a.tab = b->d_small;
    a.Nmax = b->Nmax;
    if (a.ntiles > 0) {
        const int G = std::min(a.ntiles, b->grid_cap);
        b->ks->init_product(a, G, sizeof(int) * (size_t)b->Tn, s);
        FH_HIP(hipGetLastError());
    }
    FH_HIP(hipStreamSynchronize(s));
    return FH_OK;
}

}  // namespace

// ===================================================================== ABI ==
extern "C" {

const char* fh_last_error(void) { return g_last_error.c_str(); }
int fh_version(void) { return 100; }

fh_status fh_model_create(int M, int pmod, const double* omega, double Lambda, const double* V, fh_model** out) {
    return Guard::run([&] { return make_model(M, pmod, omega, Lambda, V, out); });
}

fh_status fh_model_transpose(const fh_model* m, fh_model** out) {
    return Guard::run([&]() -> fh_status {
        FH_REQUIRE(m != nullptr, FH_EINVAL, "fh_model_transpose: model is NULL");
        const int M = m->M;
        std::vector<double> VT(m->V.size());
        for (int i = 0; i < M; ++i)
            for (int j = 0; j < M; ++j)
                for (int k = 0; k < M; ++k)
                    for (int l = 0; l < M; ++l)
                        VT[(((size_t)i * M + j) * M + k) * M + l] = m->V[(((size_t)k * M + l) * M + i) * M + j];
        return make_model(M, m->pmod, m->omega.data(), m->Lambda, VT.data(), out);
    });
}

fh_status fh_model_destroy(fh_model* m) {
    if (m) {
        (void)hipFree(m->d_coef);
        delete m;
    }
    return FH_OK;
}

fh_status fh_basis_create(int M, int pmod, int nsec, const int32_t* N, const int32_t* P, fh_basis** out) {
    return Guard::run([&] { return make_basis(M, pmod, nsec, N, P, out); });
}

fh_status fh_basis_destroy(fh_basis* b) {
    basis_free(b);
    return FH_OK;
}

fh_status fh_basis_info(const fh_basis* b, int* M, int* pmod, int* nsec, int64_t* total) {
    FH_REQUIRE(b != nullptr, FH_EINVAL, "fh_basis_info: basis is NULL");
    if (M) *M = b->M;
    if (pmod) *pmod = b->pmod;
    if (nsec) *nsec = b->nsec;
    if (total) *total = b->total;
    return FH_OK;
}

fh_status fh_basis_sizes(const fh_basis* b, int64_t* dim, int64_t* offset) {
    FH_REQUIRE(b != nullptr, FH_EINVAL, "fh_basis_sizes: basis is NULL");
    if (dim) std::copy(b->dim.begin(), b->dim.end(), dim);
    if (offset) std::copy(b->off.begin(), b->off.end(), offset);
    return FH_OK;
}

fh_status fh_basis_set_launch(fh_basis* b, int blocks_per_cu, int xcd_order) {
    FH_REQUIRE(b != nullptr, FH_EINVAL, "fh_basis_set_launch: basis is NULL");
    FH_REQUIRE(blocks_per_cu >= 0 && blocks_per_cu <= 8, FH_EINVAL, "blocks_per_cu must be in [0, 8]");
    FH_REQUIRE(xcd_order >= 0 && xcd_order <= 3, FH_EINVAL, "xcd_order must be 0, 1, 2 or 3");
    b->blocks_per_cu = blocks_per_cu;
    b->xcd_order = xcd_order;
    return FH_OK;
}

fh_status fh_basis_set_tile_order(fh_basis* b, int order, int prefix_modes) {
    return Guard::run([&]() -> fh_status {
        FH_REQUIRE(b != nullptr, FH_EINVAL, "fh_basis_set_tile_order: basis is NULL");
        FH_REQUIRE(order == 0 || order == 1, FH_EINVAL, "fh_basis_set_tile_order: order must be 0 or 1");
        FH_REQUIRE(prefix_modes >= 0 && prefix_modes <= std::min(b->M - 1, 8), FH_EINVAL,
                   "fh_basis_set_tile_order: prefix_modes must be in [0, min(M-1, 8)]");
        const int M = b->M, p = b->pmod, h = prefix_modes;
        std::vector<Tile> tiles;
        std::vector<int> begin(b->nsec + 1);
        for (int s = 0; s < b->nsec; ++s) {
            begin[s] = (int)tiles.size();
            // Blocks: rows sharing the occupations of modes 0..h-1 are
            // contiguous in lexicographic order; walk the prefixes in that
            // order, with block sizes D_h(remaining bosons, remaining momentum).
            std::vector<std::pair<uint64_t, Tile>> keyed;
            std::vector<int> pre(std::max(h, 1), 0);
            int64_t start = 0;
            auto emit = [&](int64_t size) {
                uint64_t key = 0;  // Morton key: interleave the bits of the prefix
                for (int bit = 7; bit >= 0; --bit)
                    for (int m = 0; m < h; ++m) key = (key << 1) | (uint64_t)((pre[m] >> bit) & 1);
                for (int64_t r = 0; r < size; r += kTileRows)
                    keyed.push_back({key, Tile{s, (int)(start + r), (int)std::min<int64_t>(kTileRows, size - r), 0}});
                start += size;
            };
            auto rec = [&](auto&& self, int m, int R, int Q) -> void {
                if (m == h) {
                    const int64_t size = b->D_at(h, R, Q);
                    if (size > 0) emit(size);
                    return;
                }
                for (int v = 0; v <= R; ++v) {
                    pre[m] = v;
                    self(self, m + 1, R - v, posmod((long long)Q - (long long)m * v, p));
                }
            };
            rec(rec, 0, b->N[s], b->P[s]);
            FH_REQUIRE(start == b->dim[s], FH_EINVAL, "fh_basis_set_tile_order: internal block count mismatch");
            if (order == 1)
                std::stable_sort(keyed.begin(), keyed.end(),
                                 [](const auto& x, const auto& y) { return x.first < y.first; });
            for (auto& kt : keyed) tiles.push_back(kt.second);
        }
        begin[b->nsec] = (int)tiles.size();
        if (tiles.size() > b->tiles.size() || b->d_tiles == nullptr) {
            Tile* d = nullptr;
            FH_HIP(hipMalloc(&d, sizeof(Tile) * std::max<size_t>(1, tiles.size())));
            FH_HIP(hipDeviceSynchronize());
            (void)hipFree(b->d_tiles);
            b->d_tiles = d;
        }
        b->tiles.swap(tiles);
        b->tile_begin.swap(begin);
        b->tile_order = order;
        b->prefix_modes = prefix_modes;
        (void)M;
        if (!b->tiles.empty())
            FH_HIP(hipMemcpy(b->d_tiles, b->tiles.data(), sizeof(Tile) * b->tiles.size(), hipMemcpyHostToDevice));
        return FH_OK;
    });
}

fh_status fh_basis_rank(const fh_basis* b, int sec, int64_t count, const uint8_t* occ, int64_t* idx, void* stream) {
    FH_REQUIRE(b != nullptr, FH_EINVAL, "fh_basis_rank: basis is NULL");
    FH_REQUIRE(sec >= 0 && sec < b->nsec, FH_EINVAL, "fh_basis_rank: sector out of range");
    FH_REQUIRE(count >= 0, FH_EINVAL, "fh_basis_rank: negative count");
    FH_REQUIRE(count == 0 || (occ && idx), FH_EINVAL, "fh_basis_rank: NULL buffer");
    RankArgs a{};
    a.occ = occ;
    a.idx = idx;
    a.count = count;
    a.N = b->N[sec];
    a.P = b->P[sec];
    a.dim = (int)b->dim[sec];
    a.T = b->d_T;
    a.Tn = b->Tn;
    a.Rdim = b->Rdim;
    b->ks->rank(a, as_stream(stream));
    FH_HIP(hipGetLastError());
    return FH_OK;
}

fh_status fh_basis_unrank(const fh_basis* b, int sec, int64_t count, const int64_t* idx, uint8_t* occ, void* stream) {
    FH_REQUIRE(b != nullptr, FH_EINVAL, "fh_basis_unrank: basis is NULL");
    FH_REQUIRE(sec >= 0 && sec < b->nsec, FH_EINVAL, "fh_basis_unrank: sector out of range");
    FH_REQUIRE(count >= 0, FH_EINVAL, "fh_basis_unrank: negative count");
    FH_REQUIRE(count == 0 || (occ && idx), FH_EINVAL, "fh_basis_unrank: NULL buffer");
    RankArgs a{};
    a.idx_in = idx;
    a.occ_out = occ;
    a.count = count;
    a.N = b->N[sec];
    a.P = b->P[sec];
    a.dim = (int)b->dim[sec];
    a.T = b->d_T;
    a.Tn = b->Tn;
    a.Rdim = b->Rdim;
    b->ks->unrank(a, as_stream(stream));
    FH_HIP(hipGetLastError());
    return FH_OK;
}

fh_status fh_basis_occupations(const fh_basis* b, uint8_t* occ, void* stream) {
    FH_REQUIRE(b != nullptr && occ != nullptr, FH_EINVAL, "fh_basis_occupations: NULL argument");
    // Reuse the unrank kernel per sector over 0..dim-1 (indices staged in the
    // partial buffer, which is large enough for a chunk of rows).
    const size_t chunk = b->partial_doubles;  // int64 slots
    std::vector<int64_t> idx;
    for (int s = 0; s < b->nsec; ++s) {
        for (int64_t r0 = 0; r0 < b->dim[s]; r0 += (int64_t)chunk) {
            const int64_t cnt = std::min<int64_t>((int64_t)chunk, b->dim[s] - r0);
            idx.resize(cnt);
            for (int64_t q = 0; q < cnt; ++q) idx[q] = r0 + q;
            FH_HIP(hipMemcpyAsync(b->d_partial, idx.data(), sizeof(int64_t) * cnt, hipMemcpyHostToDevice,
                                  as_stream(stream)));
            fh_status st = fh_basis_unrank(b, s, cnt, reinterpret_cast<const int64_t*>(b->d_partial),
                                           occ + (size_t)(b->off[s] + r0) * b->M, stream);
            if (st != FH_OK) return st;
            FH_HIP(hipStreamSynchronize(as_stream(stream)));
        }
    }
    return FH_OK;
}

fh_status fh_init_number(const fh_basis* b, const uint8_t* occ, int nrhs, fh_c64* psi, void* stream) {
    FH_REQUIRE(b != nullptr && occ != nullptr && psi != nullptr, FH_EINVAL, "fh_init_number: NULL argument");
    FH_REQUIRE(!bad_nrhs(nrhs), FH_EINVAL, "nrhs must be 1, 2, 4, 8 or 16");
    int Nn = 0;
    long long mom = 0;
    for (int m = 0; m < b->M; ++m) {
        Nn += occ[m];
        mom += (long long)m * occ[m];
    }
    const int Pn = posmod(mom, b->pmod);
    int sec = -1;
    for (int s = 0; s < b->nsec; ++s)
        if (b->N[s] == Nn && b->P[s] == Pn) sec = s;
    FH_REQUIRE(sec >= 0, FH_EINVAL, "fh_init_number: occupation vector lies in no retained sector");
    const int64_t r = host_rank(b, sec, occ);
    hipStream_t s = as_stream(stream);
    launch_fill(reinterpret_cast<double*>(psi), 2 * b->total * nrhs, 0.0, s);
    for (int q = 0; q < nrhs; ++q)
        launch_set_c64(reinterpret_cast<double*>(psi), (b->off[sec] + r) * nrhs + q, 1.0, 0.0, s);
    FH_HIP(hipGetLastError());
    return FH_OK;
}

fh_status fh_init_coherent(const fh_basis* b, const fh_c64* alpha, int nrhs, fh_c64* psi, void* stream) {
    return Guard::run([&]() -> fh_status {
        FH_REQUIRE(b != nullptr && alpha != nullptr && psi != nullptr, FH_EINVAL, "fh_init_coherent: NULL argument");
        FH_REQUIRE(!bad_nrhs(nrhs), FH_EINVAL, "nrhs must be 1, 2, 4, 8 or 16");
        const int M = b->M, W = b->Nmax + 1;
        std::vector<double> tab((size_t)nrhs * M * W * 2);
        for (int q = 0; q < nrhs; ++q)
            for (int m = 0; m < M; ++m) {
                const std::complex<double> a(alpha[q * M + m].re, alpha[q * M + m].im);
                FH_REQUIRE(std::isfinite(a.real()) && std::isfinite(a.imag()), FH_EINVAL, "alpha not finite");
                std::complex<double> t = std::exp(-0.5 * std::norm(a));
                for (int n = 0; n < W; ++n) {
                    if (n > 0) t = t * a / std::sqrt((double)n);
                    tab[(((size_t)q * M + m) * W + n) * 2] = t.real();
                    tab[(((size_t)q * M + m) * W + n) * 2 + 1] = t.imag();
                }
            }
        return init_product(b, nrhs, tab, reinterpret_cast<double*>(psi), as_stream(stream));
    });
}

fh_status fh_init_fieldnumber(const fh_basis* b, const fh_c64* z, int nrhs, fh_c64* psi, void* stream) {
    return Guard::run([&]() -> fh_status {
        FH_REQUIRE(b != nullptr && z != nullptr && psi != nullptr, FH_EINVAL, "fh_init_fieldnumber: NULL argument");
        FH_REQUIRE(!bad_nrhs(nrhs), FH_EINVAL, "nrhs must be 1, 2, 4, 8 or 16");
        const int M = b->M, W = b->Nmax + 1;
        std::vector<double> tab((size_t)nrhs * M * W * 2);
        for (int q = 0; q < nrhs; ++q)
            for (int m = 0; m < M; ++m) {
                const std::complex<double> a(z[q * M + m].re, z[q * M + m].im);
                FH_REQUIRE(std::isfinite(a.real()) && std::isfinite(a.imag()), FH_EINVAL, "z not finite");
                std::complex<double> t = 1.0;
                for (int n = 0; n < W; ++n) {
                    if (n > 0) t = t * a / std::sqrt((double)n);
                    tab[(((size_t)q * M + m) * W + n) * 2] = t.real();
                    tab[(((size_t)q * M + m) * W + n) * 2 + 1] = t.imag();
                }
            }
        hipStream_t s = as_stream(stream);
        fh_status st = init_product(b, nrhs, tab, reinterpret_cast<double*>(psi), s);
        if (st != FH_OK) return st;
        std::vector<double> scale(nrhs);
        std::vector<double> rec(FH_MOMENT_DOUBLES(M));
        for (int q = 0; q < nrhs; ++q) {
            st = run_moments(b, nrhs, q, reinterpret_cast<const double*>(psi), rec.data(), s, 1);
            if (st != FH_OK) return st;
            FH_REQUIRE(rec[0] > 0.0, FH_ESTATE, "fh_init_fieldnumber: state vanishes on the retained sectors");
            scale[q] = 1.0 / std::sqrt(rec[0]);
        }
        FH_HIP(hipMemcpyAsync(b->d_small, scale.data(), sizeof(double) * nrhs, hipMemcpyHostToDevice, s));
        launch_scale_rhs(reinterpret_cast<double*>(psi), b->total, nrhs, b->d_small, s);
        FH_HIP(hipGetLastError());
        FH_HIP(hipStreamSynchronize(s));
        return FH_OK;
    });
}

fh_status fh_apply_h(const fh_model* m, const fh_basis* b, int nrhs, const fh_c64* psi, fh_c64* out, void* stream) {
    return Guard::run([&]() -> fh_status {
        if (!check_model_basis(m, b)) return FH_EINVAL;
        FH_REQUIRE(!bad_nrhs(nrhs), FH_EINVAL, "nrhs must be 1, 2, 4, 8 or 16");
        FH_REQUIRE(psi != nullptr && out != nullptr, FH_EINVAL, "fh_apply_h: NULL buffer");
        FH_REQUIRE((const void*)psi != (const void*)out, FH_EINVAL, "fh_apply_h: psi and out alias");
        StageArgs a = stage_base(m, b);
        a.x = reinterpret_cast<const double*>(psi);
        a.out = reinterpret_cast<double*>(out);
        a.mode = kApply;
        return launch_stage(b, nrhs, a, 0, as_stream(stream), nullptr);
    });
}

fh_status fh_classical_rk4(const fh_model* m, int ntraj, fh_c64* alpha, double dt, int64_t nsteps, int64_t every,
                           fh_c64* out, void* stream) {
    return Guard::run([&]() -> fh_status {
        FH_REQUIRE(m != nullptr, FH_EINVAL, "fh_classical_rk4: model is NULL");
        FH_REQUIRE(ntraj >= 0 && nsteps >= 0, FH_EINVAL, "fh_classical_rk4: ntraj and nsteps must be >= 0");
        FH_REQUIRE(std::isfinite(dt), FH_EINVAL, "fh_classical_rk4: dt not finite");
        FH_REQUIRE(out == nullptr || every >= 1, FH_EINVAL, "fh_classical_rk4: every must be >= 1 with out");
        if (ntraj == 0) return FH_OK;
        FH_REQUIRE(alpha != nullptr, FH_EINVAL, "fh_classical_rk4: alpha is NULL");
        ClassicalArgs a{};
        a.alpha = reinterpret_cast<double*>(alpha);
        a.out = reinterpret_cast<double*>(out);
        a.omega = m->d_coef;
        a.U = m->d_coef + m->ucoef_off;
        a.dt = dt;
        a.nsteps = nsteps;
        a.every = out ? every : 1;
        a.ntraj = ntraj;
        kernel_set(m->M)->classical(a, as_stream(stream));
        FH_HIP(hipGetLastError());
        return FH_OK;
    });
}

fh_status fh_basis_autotune(const fh_model* m, fh_basis* b, int nrhs, const fh_c64* x, fh_c64* out,
                            const char* cache_path, int* chosen, double* best_ms, void* stream) {
    return Guard::run([&]() -> fh_status {
        if (!check_model_basis(m, b)) return FH_EINVAL;
        FH_REQUIRE(!bad_nrhs(nrhs), FH_EINVAL, "nrhs must be 1, 2, 4, 8 or 16");
        FH_REQUIRE(x != nullptr && out != nullptr && (const void*)x != (const void*)out, FH_EINVAL,
                   "fh_basis_autotune: need distinct x and out buffers");
        hipStream_t s = as_stream(stream);
        hipDeviceProp_t prop;
        FH_HIP(hipGetDeviceProperties(&prop, b->device));
        const std::string key = std::string(prop.gcnArchName) + "/cu" + std::to_string(b->num_cu) + "/M" +
                                std::to_string(b->M) + "/nrhs" + std::to_string(nrhs) + "/sec" +
                                std::to_string(b->nsec) + "/states" + std::to_string(b->total) + "/Nmax" +
                                std::to_string(b->Nmax);
        int cfg[4] = {0, 1, 0, 0};  // blocks per CU, XCD order, tile order, prefix modes
        double best = -1.0;
        bool cached = false;
        if (cache_path) {
            if (FILE* f = std::fopen(cache_path, "r")) {
                char line[512];
                while (std::fgets(line, sizeof line, f)) {
                    char k[400];
                    int c0, c1, c2, c3;
                    double ms;
                    if (std::sscanf(line, "%399s %d %d %d %d %lf", k, &c0, &c1, &c2, &c3, &ms) == 6 && key == k) {
                        cfg[0] = c0; cfg[1] = c1; cfg[2] = c2; cfg[3] = c3;
                        best = ms;
                        cached = true;
                    }
                }
                std::fclose(f);
            }
        }
        StageArgs a = stage_base(m, b);
        a.x = reinterpret_cast<const double*>(x);
        a.out = reinterpret_cast<double*>(out);
        a.mode = kApply;
        auto apply_cfg = [&](const int* c) -> fh_status {
            b->blocks_per_cu = c[0];
            b->xcd_order = c[1];
            if (b->tile_order != c[2] || b->prefix_modes != c[3]) return fh_basis_set_tile_order(b, c[2], c[3]);
            return FH_OK;
        };
        if (!cached) {
            struct Events {  // destroyed on every return path
                hipEvent_t e0 = nullptr, e1 = nullptr;
                ~Events() {
                    if (e0) (void)hipEventDestroy(e0);
                    if (e1) (void)hipEventDestroy(e1);
                }
            } ev;
            FH_HIP(hipEventCreate(&ev.e0));
            FH_HIP(hipEventCreate(&ev.e1));
            hipEvent_t e0 = ev.e0, e1 = ev.e1;
            std::vector<std::array<int, 4>> cands;
            const int maxp = std::min(b->M - 1, 3);
            for (int bpc : {0, 1, 2, 3})
                for (int xo : {3, 2, 1, 0})
                    for (int pre = 0; pre <= maxp; ++pre) {
                        if (pre == 1) continue;  // a one-mode prefix never pays
                        cands.push_back({bpc, xo, pre > 0 ? 1 : 0, pre});
                    }
            fh_status st = FH_OK;
            for (const auto& c : cands) {
                if ((st = apply_cfg(c.data())) != FH_OK) break;
                StageArgs ac = a;
                ac.xcd_order = b->xcd_order;
                if ((st = launch_stage(b, nrhs, ac, 0, s, nullptr)) != FH_OK) break;  // warm-up
                float t = 0.f, tmin = 1e30f;
                const int reps = best > 50.0 ? 1 : 3;
                for (int r = 0; r < reps; ++r) {
                    FH_HIP(hipEventRecord(e0, s));
                    if ((st = launch_stage(b, nrhs, ac, 0, s, nullptr)) != FH_OK) break;
                    FH_HIP(hipEventRecord(e1, s));
                    FH_HIP(hipEventSynchronize(e1));
                    FH_HIP(hipEventElapsedTime(&t, e0, e1));
                    tmin = std::min(tmin, t);
                }
                if (st != FH_OK) break;
                if (best < 0 || tmin < best) {
                    best = tmin;
                    std::copy(c.begin(), c.end(), cfg);
                }
            }
            if (st != FH_OK) return st;
            if (cache_path) {
                if (FILE* f = std::fopen(cache_path, "a")) {
                    std::fprintf(f, "%s %d %d %d %d %.6f\n", key.c_str(), cfg[0], cfg[1], cfg[2], cfg[3], best);
                    std::fclose(f);
                }
            }
        }
        fh_status st = apply_cfg(cfg);
        if (st != FH_OK) return st;
        if (chosen) std::copy(cfg, cfg + 4, chosen);
        if (best_ms) *best_ms = best;
        return FH_OK;
    });
}

fh_status fh_moments(const fh_basis* b, int nrhs, int rhs, const fh_c64* psi, double* norm2, fh_c64* a, fh_c64* Mij,
                     fh_c64* Akl, void* stream) {
    return Guard::run([&]() -> fh_status {
        FH_REQUIRE(b != nullptr && psi != nullptr, FH_EINVAL, "fh_moments: NULL argument");
        FH_REQUIRE(!bad_nrhs(nrhs), FH_EINVAL, "nrhs must be 1, 2, 4, 8 or 16");
        FH_REQUIRE(rhs >= 0 && rhs < nrhs, FH_EINVAL, "fh_moments: rhs out of range");
        const int M = b->M;
        std::vector<double> rec(FH_MOMENT_DOUBLES(M));
        const int groups = (Mij || Akl) ? M + 1 : 1;
        fh_status st = run_moments(b, nrhs, rhs, reinterpret_cast<const double*>(psi), rec.data(), as_stream(stream),
                                   groups);
        if (st != FH_OK) return st;
        if (norm2) *norm2 = rec[0];
        if (a) std::memcpy(a, rec.data() + 1, sizeof(double) * 2 * M);
        if (Mij) std::memcpy(Mij, rec.data() + 1 + 2 * M, sizeof(double) * 2 * M * M);
        if (Akl) std::memcpy(Akl, rec.data() + 1 + 2 * M + 2 * M * M, sizeof(double) * 2 * M * M);
        return FH_OK;
    });
}

}  // extern "C"

namespace {

// Shared driver of the explicit steppers: one step is the given sequence of
// fused stage launches (buffers already bound); moments every obs_every steps;
// optionally the step is captured once into a HIP graph and replayed.
fh_status evolve_driver(const fh_basis* b, int nrhs, double* P, std::vector<StageArgs>& stages, int64_t nsteps,
                        int64_t obs_every, double* moments, int64_t moments_capacity, int flags, fh_timing* timing,
                        hipStream_t s, std::chrono::steady_clock::time_point t0, const char* who) {
    const int M = b->M;
    const int64_t nrec = obs_every > 0 ? nsteps / obs_every + 1 : 0;
    const int64_t per = (int64_t)FH_MOMENT_DOUBLES(M) * nrhs;
    if (nrec > 0) {
        FH_REQUIRE(moments != nullptr, FH_EINVAL, std::string(who) + ": moments buffer is NULL");
        FH_REQUIRE(moments_capacity >= nrec * per, FH_ENOMEM, std::string(who) + ": moments buffer too small");
    }
    StageTimer tm;
    fh_status st = tm.init((flags & FH_TIMING) != 0, s);
    if (st != FH_OK) return st;
    StageTimer* tmp = (flags & FH_TIMING) ? &tm : nullptr;

    auto record = [&](int64_t r) -> fh_status {
        for (int q = 0; q < nrhs; ++q) {
            fh_status e = run_moments(b, nrhs, q, P, moments + r * per + (int64_t)q * FH_MOMENT_DOUBLES(M), s, M + 1);
            if (e != FH_OK) return e;
        }
        return FH_OK;
    };
    auto step_direct = [&]() -> fh_status {
        for (StageArgs& a : stages) {
            fh_status e = launch_stage(b, nrhs, a, flags, s, tmp);
            if (e != FH_OK) return e;
        }
        return FH_OK;
    };

    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    if (flags & FH_GRAPH) {
        FH_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        fh_status e = step_direct();
        hipError_t ce = hipStreamEndCapture(s, &graph);
        if (e != FH_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return e;
        }
        if (ce != hipSuccess) return hip_fail(ce, "hipStreamEndCapture");
        hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (ie != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return hip_fail(ie, "hipGraphInstantiate");
        }
    }
    auto cleanup = [&]() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    };

    int64_t r = 0;
    if (nrec > 0) {
        st = record(r++);
        if (st != FH_OK) { cleanup(); return st; }
    }
    for (int64_t step = 1; step <= nsteps; ++step) {
        if (exec) {
            hipError_t e = hipGraphLaunch(exec, s);
            if (e != hipSuccess) { cleanup(); return hip_fail(e, "hipGraphLaunch"); }
        } else {
            st = step_direct();
            if (st != FH_OK) { cleanup(); return st; }
        }
        if (obs_every > 0 && step % obs_every == 0) {
            st = record(r++);
            if (st != FH_OK) { cleanup(); return st; }
        }
    }
    cleanup();
    st = tm.flush();
    if (st != FH_OK) return st;
    FH_HIP(hipStreamSynchronize(s));
    if (timing) {
        timing->stage_ms = tm.ms;
        timing->stage_launches = tm.launches;
        timing->wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    for (int64_t q = 0; q < nrec * per; q += FH_MOMENT_DOUBLES(M))
        if (!std::isfinite(moments[q])) {
            set_error(std::string(who) + ": non-finite norm (unstable dt?)");
            return FH_ESTATE;
        }
    return FH_OK;
}

fh_status check_evolve_args(const fh_model* m, const fh_basis* b, int nrhs, const fh_c64* psi, const fh_c64* work,
                            double dt, int64_t nsteps, int64_t obs_every, int flags, void* stream, const char* who) {
    if (!check_model_basis(m, b)) return FH_EINVAL;
    const std::string w(who);
    FH_REQUIRE(!bad_nrhs(nrhs), FH_EINVAL, "nrhs must be 1, 2, 4, 8 or 16");
    FH_REQUIRE(psi != nullptr && work != nullptr, FH_EINVAL, w + ": NULL buffer");
    FH_REQUIRE(nsteps >= 0 && obs_every >= 0, FH_EINVAL, w + ": negative step count");
    FH_REQUIRE(std::isfinite(dt), FH_EINVAL, w + ": dt not finite");
    FH_REQUIRE(!((flags & FH_GRAPH) && (flags & FH_TIMING)), FH_EINVAL, "FH_GRAPH and FH_TIMING are exclusive");
    FH_REQUIRE(!((flags & FH_GRAPH) && stream == nullptr), FH_EINVAL, "FH_GRAPH needs a non-default stream");
    return FH_OK;
}

}  // namespace

extern "C" {

fh_status fh_evolve_rk4(const fh_model* m, const fh_basis* b, int nrhs, fh_c64* psi, fh_c64* work, double dt,
                        int64_t nsteps, int64_t obs_every, double* moments, int64_t moments_capacity, int flags,
                        fh_timing* timing, void* stream) {
    return Guard::run([&]() -> fh_status {
        const auto t0 = std::chrono::steady_clock::now();
        fh_status st = check_evolve_args(m, b, nrhs, psi, work, dt, nsteps, obs_every, flags, stream, "fh_evolve_rk4");
        if (st != FH_OK) return st;
        double* P = reinterpret_cast<double*>(psi);
        const int64_t vec = 2 * b->total * nrhs;
        double* acc = reinterpret_cast<double*>(work);
        double* yA = acc + vec;
        double* yB = yA + vec;
        StageArgs base = stage_base(m, b);
        base.ks_re = 0.0;
        base.ks_im = -1.0;
        StageArgs s1 = base, s2 = base, s3 = base, s4 = base;
        s1.x = P; s1.base = P; s1.acc = acc; s1.ynext = yA; s1.mode = kFirst; s1.a = dt / 6; s1.c0 = 1; s1.b = dt / 2;
        s2.x = yA; s2.base = P; s2.acc = acc; s2.ynext = yB; s2.mode = kMid; s2.a = dt / 3; s2.c0 = 1; s2.b = dt / 2;
        s3.x = yB; s3.base = P; s3.acc = acc; s3.ynext = yA; s3.mode = kMid; s3.a = dt / 3; s3.c0 = 1; s3.b = dt;
        s4.x = yA; s4.acc = acc; s4.baseout = P; s4.mode = kLast; s4.a = dt / 6;
        std::vector<StageArgs> stages = {s1, s2, s3, s4};
        return evolve_driver(b, nrhs, P, stages, nsteps, obs_every, moments, moments_capacity, flags, timing,
                             as_stream(stream), t0, "fh_evolve_rk4");
    });
}

fh_status fh_evolve_taylor2(const fh_model* m, const fh_basis* b, int nrhs, fh_c64* psi, fh_c64* work, double dt,
                            double c2, int64_t nsteps, int64_t obs_every, double* moments, int64_t moments_capacity,
                            int flags, fh_timing* timing, void* stream) {
    return Guard::run([&]() -> fh_status {
        const auto t0 = std::chrono::steady_clock::now();
        fh_status st =
            check_evolve_args(m, b, nrhs, psi, work, dt, nsteps, obs_every, flags, stream, "fh_evolve_taylor2");
        if (st != FH_OK) return st;
        FH_REQUIRE(std::isfinite(c2), FH_EINVAL, "fh_evolve_taylor2: c2 not finite");
        double* P = reinterpret_cast<double*>(psi);
        const int64_t vec = 2 * b->total * nrhs;
        double* acc = reinterpret_cast<double*>(work);
        double* y = acc + vec;
        // stage A: k = -i dt H psi;        acc = psi + k,  y = k
        // stage B: k = -i c2 dt H y;       psi = acc + k = psi - i dt H psi - c2 dt^2 H^2 psi
        StageArgs sa = stage_base(m, b), sb = sa;
        sa.x = P; sa.base = P; sa.acc = acc; sa.ynext = y; sa.mode = kFirst;
        sa.ks_re = 0.0; sa.ks_im = -dt; sa.a = 1.0; sa.c0 = 0.0; sa.b = 1.0;
        sb.x = y; sb.acc = acc; sb.baseout = P; sb.mode = kLast;
        sb.ks_re = 0.0; sb.ks_im = -c2 * dt; sb.a = 1.0;
        std::vector<StageArgs> stages = {sa, sb};
        return evolve_driver(b, nrhs, P, stages, nsteps, obs_every, moments, moments_capacity, flags, timing,
                             as_stream(stream), t0, "fh_evolve_taylor2");
    });
}

}  // extern "C"

// ================================================================ adjoint ==
namespace {

int max_class_size(int M) {
    int best = 0;
    for (int c = 0; c < M; ++c) {
        int n = 0;
        for (int i = 0; i < M; ++i)
            for (int j = i; j < M; ++j)
                if ((i + j) % M == c) ++n;
        best = std::max(best, n);
    }
    return best;
}

// Member index of pair {i,j} inside its class (pair order).
int class_rank(int M, int i, int j) {
    if (i > j) std::swap(i, j);
    const int c = (i + j) % M;
    int r = 0;
    for (int a = 0; a < M; ++a)
        for (int b = a; b < M; ++b)
            if ((a + b) % M == c) {
                if (a == i && b == j) return r;
                ++r;
            }
    return -1;
}

// Workgroups per momentum class of a correlator launch (grid Gc x M,
// blockIdx.y the class), from the resident grid G of the launch.  A long
// launch (at least 16 tiles per resident workgroup) gives every class all of G,
// so that the classes run one after another and each sweep's gather footprint
// is that of one class's moves (running them side by side was slower there:
// the 55.5M-state M = 6 adjoint took 3.67 instead of 3.44 forward runs).  A
// short launch gives each class G / M (at most one per tile), so that all
// classes run at once and every workgroup takes several tiles and stages its
// tables once for them (with one workgroup per tile and class most of them
// waited for a slot: the 54k-state M = 6 adjoint took 3.45 forward runs, now
// 2.73).
int corr_class_grid(int M, int G, int ntiles) {
    if ((long long)ntiles >= 16LL * G) return G;
    return std::max(1, std::min(ntiles, G / M));
}

// Rows per correlator launch where the classes walk statically (run_corr).
constexpr long long kCorrChunkRows = 1LL << 24;

// gtotal += correlators of the kCorrPairs pairs (uscale[q] u[q], y[q]) for column rhs.
// With several columns and at least 2 x (pairs per launch) single-column
// buffers in colbuf, each launch's u and y columns are first copied out
// contiguous and the launch runs as for one column (its buffer-load gathers
// then read whole lines of the one column instead of every nrhs-th 16 bytes;
// the launches and their sums are those of a one-column run, bit for bit).
fh_status run_corr(const fh_basis* b, int nrhs, int rhs, const double* const (&u)[kCorrPairs],
                   const double (&uscale)[kCorrPairs], const double* const (&y)[kCorrPairs], double* gtotal,
                   hipStream_t s, double* const* colbuf = nullptr, int ncolbuf = 0) {
    const int nt = (int)b->tiles.size();
    if (nt == 0) return FH_OK;
    const int M = b->M;
    const int NV = 2 * max_class_size(M) * max_class_size(M);
    const size_t lds = lds_bytes(b, 4 * NV);
    CorrArgs a{};
    a.nrhs = nrhs;
    a.rhs = rhs;
    a.T = b->d_T;
    a.Tn = b->Tn;
    a.Rdim = b->Rdim;
    a.sqrt_tab = b->d_sqrt;
    a.nsqrt = (int)b->sqrt_tab.size();
    a.tiles = b->d_tiles;
    a.ntiles = nt;
    a.secs = b->d_secs;
    a.partial = b->d_partial;
    a.xcd_order = b->xcd_order;
    a.occ = b->d_occ;
    const int G = corr_class_grid(M, persistent_grid(b, b->ks->corr_fn, lds, nt * M), nt);
    // the correlator kernel takes its tiles from the counters at M <= 7 only
    a.queue = M <= 7 && use_queue(b, nt, G) ? b->d_queue : nullptr;
    // Where the classes walk their tiles statically (M >= 8), a launch covers
    // the tiles of 2^24 rows at a time, its classes one after another over
    // them, so that the classes' sweeps over the same rows (their records, u
    // and y, and their gather windows) sit close together in time (the M = 10
    // adjoint: 7.53 -> 6.93 s; chunks of 1e6 rows: 8.06 s, of 6.4e7 rows:
    // 7.18 s).  Under the counter walk (M <= 7) one launch covers all tiles (at
    // M = 6 chunks were slower, 6.16 -> 6.25 s).
    const int tchunk = M >= 8 ? std::max(1, (int)(kCorrChunkRows / kTileRows)) : nt;
    const int per = corr_pairs_per_launch(M);
    const bool take = nrhs > 1 && colbuf != nullptr && ncolbuf >= 2 * per;
    if (take) {
        a.nrhs = 1;
        a.rhs = 0;
    }
    for (int p0 = 0; p0 < kCorrPairs; p0 += per) {
        for (int q = 0; q < per; ++q) {
            a.u[q] = u[p0 + q];
            a.y[q] = y[p0 + q];
            a.uscale[q] = uscale[p0 + q];
            if (take) {
                launch_take_column(u[p0 + q], colbuf[q], b->total, nrhs, rhs, s);
                launch_take_column(y[p0 + q], colbuf[per + q], b->total, nrhs, rhs, s);
                FH_HIP(hipGetLastError());
                a.u[q] = colbuf[q];
                a.y[q] = colbuf[per + q];
            }
        }
        for (int t0 = 0; t0 < nt; t0 += tchunk) {
            a.tiles = b->d_tiles + t0;
            a.ntiles = std::min(tchunk, nt - t0);
            if (a.queue) {
                launch_fill(reinterpret_cast<double*>(b->d_queue), 4 * M, 0.0, s);  // counters [class][XCD] = 0
                FH_HIP(hipGetLastError());
            }
            b->ks->corr(a, G, M, lds, s);  // one row of workgroups per momentum class
            FH_HIP(hipGetLastError());
            launch_reduce_partials(b->d_partial, M, G, 2 * kCorrOutMax, 2 * kCorrOutMax, gtotal, 1, s);
            FH_HIP(hipGetLastError());
        }
    }
    return FH_OK;
}

fh_status run_onebody(const fh_basis* b, int nrhs, int rhs, const double* psi, double* out,
                      const std::vector<double>& cf, hipStream_t s) {
    const int nt = (int)b->tiles.size();
    if (nt == 0) return FH_OK;
    double* dcf = b->d_small + (b->small_doubles - 8192);
    FH_REQUIRE(cf.size() <= 8192, FH_EUNSUPPORTED, "one-body coefficient table too large");
    FH_HIP(hipMemcpyAsync(dcf, cf.data(), sizeof(double) * cf.size(), hipMemcpyHostToDevice, s));
    OneBodyArgs a{};
    a.psi = psi;
    a.out = out;
    a.nrhs = nrhs;
    a.rhs = rhs;
    a.T = b->d_T;
    a.Tn = b->Tn;
    a.Rdim = b->Rdim;
    a.sqrt_tab = b->d_sqrt;
    a.nsqrt = (int)b->sqrt_tab.size();
    a.tiles = b->d_tiles;
    a.ntiles = nt;
    a.secs = b->d_secs;
    a.secmap = b->d_secmap;
    a.Nmax = b->Nmax;
    a.cf = dcf;
    const size_t lds = lds_bytes(b, 0);
    const int G = persistent_grid(b, b->ks->onebody_fn, lds, nt);
    b->ks->onebody(a, G, lds, s);
    FH_HIP(hipGetLastError());
    // cf is a host vector that dies on return: make the upload complete first.
    FH_HIP(hipStreamSynchronize(s));
    return FH_OK;
}

// Terminal value J and the coefficients of g_T = 2 dJ/d conj(psi_T) in the
// one-body form c0 x + cN N x + sum u_i a_i x + sum v_i a_i^+ x + sum h_ij a_i^+ a_j x.
fh_status terminal_coefficients(int M, const double* rec, int objective, int obj_mode, double* J,
                                std::vector<double>& cf) {
    using cd = std::complex<double>;
    const double nu = rec[0];
    FH_REQUIRE(nu > 0.0 && std::isfinite(nu), FH_ESTATE, "adjoint: terminal state has zero or non-finite norm");
    cf.assign(4 + 4 * M + 2 * M * M, 0.0);
    auto setc = [&](int idx, cd v) {
        cf[2 * idx] = v.real();
        cf[2 * idx + 1] = v.imag();
    };
    std::vector<cd> a(M);
    for (int i = 0; i < M; ++i) a[i] = cd(rec[1 + 2 * i], rec[2 + 2 * i]) / nu;
    const double* rM = rec + 1 + 2 * M;
    double n = 0.0;
    for (int i = 0; i < M; ++i) n += rM[2 * (i * M + i)] / nu;
    FH_REQUIRE(n > 0.0, FH_ESTATE, "adjoint: terminal state has no particles");
    if (objective == FH_J_Q) {
        double S = 0.0;
        for (int i = 0; i < M; ++i) S += std::norm(a[i]);
        *J = 1.0 - S / n;
        setc(0, 2.0 * S / (n * nu));
        setc(1, 2.0 * S / (n * n * nu));
        for (int i = 0; i < M; ++i) {
            setc(2 + i, -2.0 * std::conj(a[i]) / (n * nu));
            setc(2 + M + i, -2.0 * a[i] / (n * nu));
        }
    } else if (objective == FH_J_PO) {
        std::vector<fh_c64> av(M), Mv(M * M), Av(M * M), xi(M);
        for (int i = 0; i < M; ++i) av[i] = fh_c64{rec[1 + 2 * i], rec[2 + 2 * i]};
        for (int q = 0; q < M * M; ++q) {
            Mv[q] = fh_c64{rM[2 * q], rM[2 * q + 1]};
            Av[q] = fh_c64{rec[1 + 2 * M + 2 * M * M + 2 * q], rec[2 + 2 * M + 2 * M * M + 2 * q]};
        }
        fh_obs_scalars sc{};
        fh_status st = fh_derive(M, nu, av.data(), Mv.data(), Av.data(), &sc, xi.data(), nullptr, nullptr, nullptr, nullptr,
                                 nullptr);
        if (st != FH_OK) return st;
        *J = 1.0 - sc.lambda_p / n;
        setc(1, 2.0 * sc.lambda_p / (n * n * nu));
        for (int i = 0; i < M; ++i)
            for (int j = 0; j < M; ++j) {
                const cd xi_i(xi[i].re, xi[i].im), xi_j(xi[j].re, xi[j].im);
                setc(2 + 2 * M + i * M + j, -2.0 * std::conj(xi_i) * xi_j / (n * nu));
            }
    } else if (objective == FH_J_NMODE) {
        FH_REQUIRE(obj_mode >= 0 && obj_mode < M, FH_EINVAL, "adjoint: obj_mode out of range");
        const double Jv = rM[2 * (obj_mode * M + obj_mode)] / nu;
        *J = Jv;
        setc(0, -2.0 * Jv / nu);
        setc(2 + 2 * M + obj_mode * M + obj_mode, 2.0 / nu);
    } else {
        set_error("adjoint: unknown objective");
        return FH_EINVAL;
    }
    return FH_OK;
}

}  // namespace

extern "C" {

int64_t fh_adjoint_work_states(int64_t nsteps, int64_t ckpt_every) {
    if (nsteps < 1 || ckpt_every < 1) return -1;
    const int64_t nseg = (nsteps + ckpt_every - 1) / ckpt_every;
    return nseg + std::min(ckpt_every, nsteps) + 10;
}

int64_t fh_adjoint_work_states_kept(int64_t nsteps, int64_t ckpt_every) {
    if (nsteps < 1 || ckpt_every < 1) return -1;
    const int64_t nseg = (nsteps + ckpt_every - 1) / ckpt_every;
    return nseg + 4 * std::min(ckpt_every, nsteps) + 10;
}

fh_status fh_adjoint_rk4(const fh_model* m, const fh_basis* b, int nrhs, const fh_c64* psi0, double dt, int64_t nsteps,
                         int64_t ckpt_every, int objective, int obj_mode, fh_c64* work, int64_t work_states,
                         fh_c64* lambda0, double* J, double* dJ_dLambda, double* dJ_dV, void* stream) {
    return Guard::run([&]() -> fh_status {
        if (!check_model_basis(m, b)) return FH_EINVAL;
        FH_REQUIRE(!bad_nrhs(nrhs), FH_EINVAL, "nrhs must be 1, 2, 4, 8 or 16");
        FH_REQUIRE(psi0 && work && lambda0 && J && dJ_dLambda, FH_EINVAL, "fh_adjoint_rk4: NULL argument");
        FH_REQUIRE(nsteps >= 1 && ckpt_every >= 1, FH_EINVAL, "fh_adjoint_rk4: nsteps and ckpt_every must be >= 1");
        FH_REQUIRE(std::isfinite(dt), FH_EINVAL, "fh_adjoint_rk4: dt not finite");
        FH_REQUIRE(objective >= FH_J_Q && objective <= FH_J_NMODE, FH_EINVAL, "fh_adjoint_rk4: unknown objective");
        const int64_t need = fh_adjoint_work_states(nsteps, ckpt_every);
        FH_REQUIRE(work_states >= need, FH_ENOMEM, "fh_adjoint_rk4: work buffer too small");
        const int M = b->M;
        hipStream_t s = as_stream(stream);
        const int64_t C = std::min(ckpt_every, nsteps);
        const int64_t nseg = (nsteps + ckpt_every - 1) / ckpt_every;
        // Segment lengths: the first segment takes the remainder and the others
        // C steps each, so that the last one (reversed first and, with kept
        // stage inputs, never recomputed) is a whole one.
        const int64_t first_len = nsteps - (nseg - 1) * C;  // in [1, C]
        auto seg_len = [&](int64_t k) { return k == 0 ? first_len : C; };
        // With room for 4 vectors per step of a segment, the stage inputs of
        // every step are kept from the segment's forward recompute instead of
        // being recomputed (3 H psi per step fewer).
        const bool keep = work_states >= fh_adjoint_work_states_kept(nsteps, ckpt_every);
        const int64_t vec = 2 * b->total * nrhs;  // doubles per state vector
        const size_t vbytes = sizeof(double) * (size_t)vec;
        double* W = reinterpret_cast<double*>(work);
        auto buf = [&](int64_t q) { return W + q * vec; };
        // layout: checkpoints [nseg] | segment states [C] | (kept) y2, y3, y4 [C each] | scratch [10]
        auto segst = [&](int64_t t) { return buf(nseg + t); };
        auto kept = [&](int which, int64_t t) { return buf(nseg + (int64_t)which * C + t); };  // which = 1..3
        const int64_t sb = nseg + (keep ? 4 * C : C);
        double* acc = buf(sb + 0);
        double* yA = buf(sb + 1);
        double* yB = buf(sb + 2);
        double* y2 = buf(sb + 3);
        double* y3 = buf(sb + 4);
        double* y4 = buf(sb + 5);
        double* gacc = buf(sb + 6);
        double* kbA = buf(sb + 7);
        double* kbB = buf(sb + 8);
        double* kbC = buf(sb + 9);
        double* g = reinterpret_cast<double*>(lambda0);

        fh_model* mT = nullptr;
        fh_status st = fh_model_transpose(m, &mT);
        if (st != FH_OK) return st;
        struct Del {
            fh_model* p;
            ~Del() { fh_model_destroy(p); }
        } del{mT};

        // One forward RK4 step from -> to (4 fused stages; to may equal from),
        // leaving the stage inputs y2, y3, y4 in the given buffers (the third
        // may alias the first).  With nstages = 3 only the stage inputs.
        auto step = [&](const double* from, double* to, double* o2, double* o3, double* o4,
                        int nstages) -> fh_status {
            StageArgs base = stage_base(m, b);
            base.ks_re = 0.0;
            base.ks_im = -1.0;
            StageArgs s1 = base, s2 = base, s3 = base, s4 = base;
            s1.x = from; s1.base = from; s1.acc = acc; s1.ynext = o2; s1.mode = kFirst; s1.a = dt / 6; s1.c0 = 1; s1.b = dt / 2;
            s2.x = o2; s2.base = from; s2.acc = acc; s2.ynext = o3; s2.mode = kMid; s2.a = dt / 3; s2.c0 = 1; s2.b = dt / 2;
            s3.x = o3; s3.base = from; s3.acc = acc; s3.ynext = o4; s3.mode = kMid; s3.a = dt / 3; s3.c0 = 1; s3.b = dt;
            s4.x = o4; s4.acc = acc; s4.baseout = to; s4.mode = kLast; s4.a = dt / 6;
            StageArgs* all[4] = {&s1, &s2, &s3, &s4};
            for (int q = 0; q < nstages; ++q) {
                fh_status e = launch_stage(b, nrhs, *all[q], 0, s, nullptr);
                if (e != FH_OK) return e;
            }
            return FH_OK;
        };

        // ---- forward sweep storing checkpoints (the running state is the
        //      first segment slot).  With kept stage inputs, the last segment
        //      (the first one reversed) keeps its states and stage inputs
        //      here, so that the reverse sweep need not recompute it.
        double* run = segst(0);
        FH_HIP(hipMemcpyAsync(buf(0), psi0, vbytes, hipMemcpyDeviceToDevice, s));
        FH_HIP(hipMemcpyAsync(run, psi0, vbytes, hipMemcpyDeviceToDevice, s));
        for (int64_t k = 0; k < nseg; ++k) {
            const int64_t len = seg_len(k);
            if (keep && k == nseg - 1) {
                // state(0) is the checkpoint buf(k) (== run); states 1..len-1 go to
                // the segment slots, psi_T to run
                for (int64_t t = 0; t < len; ++t) {
                    const double* from = t == 0 ? buf(k) : segst(t);
                    double* to = t + 1 < len ? segst(t + 1) : run;
                    st = step(from, to, kept(1, t), kept(2, t), kept(3, t), 4);
                    if (st != FH_OK) return st;
                }
                break;
            }
            for (int64_t t = 0; t < len; ++t) {
                st = step(run, run, yA, yB, yA, 4);
                if (st != FH_OK) return st;
            }
            if (k + 1 < nseg) FH_HIP(hipMemcpyAsync(buf(k + 1), run, vbytes, hipMemcpyDeviceToDevice, s));
        }
        double* seg0 = run;  // psi_T
        // ---- terminal condition (seg0 holds psi_T)
        std::vector<double> rec(FH_MOMENT_DOUBLES(M));
        std::vector<double> cf;
        for (int q = 0; q < nrhs; ++q) {
            st = run_moments(b, nrhs, q, seg0, rec.data(), s, M + 1);
            if (st != FH_OK) return st;
            st = terminal_coefficients(M, rec.data(), objective, obj_mode, &J[q], cf);
            if (st != FH_OK) return st;
            st = run_onebody(b, nrhs, q, seg0, g, cf, s);
            if (st != FH_OK) return st;
        }
        // ---- correlator accumulators, one block per rhs
        const size_t gt_per = (size_t)M * 2 * kCorrOutMax;
        double* gtot = b->d_small;
        FH_REQUIRE(gt_per * nrhs + 8192 <= b->small_doubles, FH_EUNSUPPORTED, "adjoint: scratch too small");
        launch_fill(gtot, (long long)(gt_per * nrhs), 0.0, s);

        // Single-column buffers for the correlators of several columns, carved
        // from scratch vectors the reverse sweep leaves free (yA and yB; with
        // kept stage inputs also y2, y3, y4): nrhs columns each.
        std::vector<double*> colbuf;
        if (nrhs > 1) {
            std::vector<double*> freev = {yA, yB};
            if (keep) freev.insert(freev.end(), {y2, y3, y4});
            for (double* v : freev)
                for (int c = 0; c < nrhs; ++c) colbuf.push_back(v + (int64_t)c * 2 * b->total);
        }

        StageArgs ab = stage_base(mT, b);
        ab.ks_re = 0.0;
        ab.ks_im = 1.0;
        ab.base = g;
        ab.acc = gacc;
        StageArgs b4 = ab, b3 = ab, b2 = ab, b1 = ab;
        b4.x = g; b4.mode = kFirst; b4.ks_im = dt / 6; b4.a = 1; b4.c0 = dt / 3; b4.b = dt; b4.ynext = kbA;
        b3.x = kbA; b3.mode = kMid; b3.a = 1; b3.c0 = dt / 3; b3.b = dt / 2; b3.ynext = kbB;
        b2.x = kbB; b2.mode = kMid; b2.a = 1; b2.c0 = dt / 6; b2.b = dt / 2; b2.ynext = kbC;
        b1.x = kbC; b1.mode = kLast; b1.a = 1; b1.baseout = g;


        for (int64_t k = nseg - 1; k >= 0; --k) {
            const int64_t len = seg_len(k);
            // state of step t of the segment: the checkpoint itself for t = 0
            auto state = [&](int64_t t) { return t == 0 ? buf(k) : segst(t); };
            // the last segment's states and stage inputs are already there
            const bool have = keep && k == nseg - 1;
            for (int64_t t = 1; t < len && !have; ++t) {
                st = keep ? step(state(t - 1), state(t), kept(1, t - 1), kept(2, t - 1), kept(3, t - 1), 4)
                          : step(state(t - 1), state(t), yA, yB, yA, 4);
                if (st != FH_OK) return st;
            }
            if (keep && !have) {
                st = step(state(len - 1), nullptr, kept(1, len - 1), kept(2, len - 1), kept(3, len - 1), 3);
                if (st != FH_OK) return st;
            }
            for (int64_t t = len - 1; t >= 0; --t) {
                double* ps = state(t);
                // stage inputs y2, y3, y4 of this step
                double* s2p = keep ? kept(1, t) : y2;
                double* s3p = keep ? kept(2, t) : y3;
                double* s4p = keep ? kept(3, t) : y4;
                if (!keep) {
                    st = step(ps, nullptr, y2, y3, y4, 3);
                    if (st != FH_OK) return st;
                }
                // reverse stages (transposed model): kb4 -> kbA, kb3 -> kbB,
                // kb2 -> kbC, then the correlators of all four stages in one
                // pass (the step's g is still intact), then the last stage.
                for (StageArgs* a : {&b4, &b3, &b2}) {
                    st = launch_stage(b, nrhs, *a, 0, s, nullptr);
                    if (st != FH_OK) return st;
                }
                {
                    const double* us[kCorrPairs] = {g, kbA, kbB, kbC};
                    const double sc[kCorrPairs] = {dt / 6, 1.0, 1.0, 1.0};
                    const double* ys[kCorrPairs] = {s4p, s3p, s2p, ps};
                    for (int q = 0; q < nrhs; ++q) {
                        st = run_corr(b, nrhs, q, us, sc, ys, gtot + q * gt_per, s, colbuf.data(),
                                      (int)colbuf.size());
                        if (st != FH_OK) return st;
                    }
                }
                st = launch_stage(b, nrhs, b1, 0, s, nullptr);
                if (st != FH_OK) return st;
            }
        }
        // ---- parameter gradients on the host
        std::vector<double> G(gt_per * nrhs);
        FH_HIP(hipMemcpyAsync(G.data(), gtot, sizeof(double) * G.size(), hipMemcpyDeviceToHost, s));
        FH_HIP(hipStreamSynchronize(s));
        const int SM = max_class_size(M);
        for (int q = 0; q < nrhs; ++q) {
            double dl = 0.0;
            for (int i = 0; i < M; ++i)
                for (int j = 0; j < M; ++j)
                    for (int k = 0; k < M; ++k)
                        for (int l = 0; l < M; ++l) {
                            const size_t vi = (((size_t)i * M + j) * M + k) * M + l;
                            double d = 0.0;
                            if ((i + j) % M == (k + l) % M) {
                                const int c = (i + j) % M;
                                const int slot = class_rank(M, i, j) * SM + class_rank(M, k, l);
                                // Re <kb, -i (Lambda/2) X y> = (Lambda/2) Im <kb|X|y>
                                const double im = G[q * gt_per + (size_t)c * 2 * kCorrOutMax + 2 * slot + 1];
                                d = 0.5 * m->Lambda * im;
                                dl += 0.5 * m->V[vi] * im;
                            }
                            if (dJ_dV) dJ_dV[(size_t)q * M * M * M * M + vi] = d;
                        }
            dJ_dLambda[q] = dl;
        }
        return FH_OK;
    });
}

fh_status fh_tangent_rk4(const fh_model* m, const fh_basis* b, int nrhs, fh_c64* psi, fh_c64* dpsi, fh_c64* work,
                         double dt, int64_t nsteps, int objective, int obj_mode, double* J, double* dJ_dLambda,
                         void* stream) {
    return Guard::run([&]() -> fh_status {
        if (!check_model_basis(m, b)) return FH_EINVAL;
        FH_REQUIRE(!bad_nrhs(nrhs), FH_EINVAL, "nrhs must be 1, 2, 4, 8 or 16");
        FH_REQUIRE(psi && dpsi && work && J && dJ_dLambda, FH_EINVAL, "fh_tangent_rk4: NULL argument");
        FH_REQUIRE(nsteps >= 0, FH_EINVAL, "fh_tangent_rk4: negative step count");
        FH_REQUIRE(std::isfinite(dt), FH_EINVAL, "fh_tangent_rk4: dt not finite");
        FH_REQUIRE(objective >= FH_J_Q && objective <= FH_J_NMODE, FH_EINVAL, "fh_tangent_rk4: unknown objective");
        const int M = b->M;
        hipStream_t s = as_stream(stream);
        const int64_t vec = 2 * b->total * nrhs;
        const long long ncplx = (long long)b->total * nrhs;
        double* P = reinterpret_cast<double*>(psi);
        double* Z = reinterpret_cast<double*>(dpsi);
        double* W = reinterpret_cast<double*>(work);
        double* acc = W;
        double* yA = W + vec;
        double* yB = W + 2 * vec;
        double* zacc = W + 3 * vec;
        double* zA = W + 4 * vec;
        double* zB = W + 5 * vec;
        double* hz = W + 6 * vec;
        double* gy = W + 7 * vec;
        // G = dH/dLambda: the interaction alone (omega = 0, Lambda = 1)
        fh_model* G = nullptr;
        {
            std::vector<double> zero(M, 0.0);
            fh_status st = make_model(M, m->pmod, zero.data(), 1.0, m->V.data(), &G);
            if (st != FH_OK) return st;
        }
        struct Del {
            fh_model* p;
            ~Del() { fh_model_destroy(p); }
        } del{G};
        StageArgs hb = stage_base(m, b), gb = stage_base(G, b);
        hb.mode = kApply;
        gb.mode = kApply;
        StageArgs base = stage_base(m, b);
        base.ks_re = 0.0;
        base.ks_im = -1.0;
        StageArgs s1 = base, s2 = base, s3 = base, s4 = base;
        s1.x = P; s1.base = P; s1.acc = acc; s1.ynext = yA; s1.mode = kFirst; s1.a = dt / 6; s1.c0 = 1; s1.b = dt / 2;
        s2.x = yA; s2.base = P; s2.acc = acc; s2.ynext = yB; s2.mode = kMid; s2.a = dt / 3; s2.c0 = 1; s2.b = dt / 2;
        s3.x = yB; s3.base = P; s3.acc = acc; s3.ynext = yA; s3.mode = kMid; s3.a = dt / 3; s3.c0 = 1; s3.b = dt;
        s4.x = yA; s4.acc = acc; s4.baseout = P; s4.mode = kLast; s4.a = dt / 6;
        // stage inputs of z: z, zA, zB, zA (as y: psi, yA, yB, yA)
        struct Zs {
            const double* zin;
            double* znext;
            int mode;
            double a, b;
        } zs[4] = {{Z, zA, kFirst, dt / 6, dt / 2}, {zA, zB, kMid, dt / 3, dt / 2}, {zB, zA, kMid, dt / 3, dt},
                   {zA, nullptr, kLast, dt / 6, 0.0}};
        StageArgs* ps[4] = {&s1, &s2, &s3, &s4};
        // Unless Lambda is tiny, the psi stage is H y into the stage's destination buffer (next,
        // or psi itself in the last stage; neither is read by that pass), G y = (H y -
        // diag(omega . n) y) / Lambda from it, and the psi update as a separate pass with the
        // fused epilogue's arithmetic: two H applications per stage instead of three.  The
        // subtraction costs about eps * max|omega . n| / |Lambda G| of relative accuracy in G y.
        // Bound max|omega . n| by Nmax max|omega_j| and |G| by Nmax^2 max|V| / 2 (every pair
        // term carries at most n(n-1) <= Nmax^2 bosons' worth of sqrt factors); when that ratio
        // would cost more than 1e-12 relative (and always at Lambda = 0), G y is an application
        // of G itself: three H applications per stage.
        bool via_h = false;
        {
            double wmax = 0.0, vmax = 0.0;
            for (double w : m->omega) wmax = std::max(wmax, std::fabs(w));
            for (double v : m->V) vmax = std::max(vmax, std::fabs(v));
            const double nmax = std::max(1, b->Nmax);
            const double kin = nmax * wmax, inter = 0.5 * nmax * nmax * vmax;
            via_h = m->Lambda != 0.0 && inter > 0.0 &&
                    std::numeric_limits<double>::epsilon() * kin <= 1e-12 * std::fabs(m->Lambda) * inter;
        }
        for (int64_t step = 0; step < nsteps; ++step) {
            for (int q = 0; q < 4; ++q) {
                StageArgs ga = gb, ha = hb;
                ga.x = ps[q]->x;  // y_s, before the psi stage overwrites any buffer
                ga.out = gy;
                ha.x = zs[q].zin;
                ha.out = hz;
                fh_status st = FH_OK;
                if (via_h) {
                    StageArgs hy = hb;
                    hy.x = ps[q]->x;
                    hy.out = ps[q]->mode == kLast ? ps[q]->baseout : ps[q]->ynext;
                    if ((st = launch_stage(b, nrhs, hy, 0, s, nullptr)) != FH_OK) return st;
                    launch_interaction_part(hy.out, hy.x, b->d_occ, occ_stride(M), M, m->d_coef, 1.0 / m->Lambda,
                                            b->total, nrhs, gy, s);
                    FH_HIP(hipGetLastError());
                    if ((st = launch_stage(b, nrhs, ha, 0, s, nullptr)) != FH_OK) return st;
                    const StageArgs& p = *ps[q];
                    launch_rk4_update(hy.out, p.base, p.acc, p.ynext, p.baseout, ncplx, p.mode, p.ks_re, p.ks_im, p.a,
                                      p.c0, p.b, s);
                    FH_HIP(hipGetLastError());
                } else {
                    if ((st = launch_stage(b, nrhs, ga, 0, s, nullptr)) != FH_OK) return st;
                    if ((st = launch_stage(b, nrhs, ha, 0, s, nullptr)) != FH_OK) return st;
                    if ((st = launch_stage(b, nrhs, *ps[q], 0, s, nullptr)) != FH_OK) return st;
                }
                launch_tangent_stage(hz, gy, Z, zacc, zs[q].znext, Z, ncplx, zs[q].mode, zs[q].a, 1.0, zs[q].b, s);
                FH_HIP(hipGetLastError());
            }
        }
        // dJ/dLambda = Re <g, z(T)> with g = 2 dJ/d conj(psi) at T (same terminal vector as the adjoint)
        std::vector<double> rec(FH_MOMENT_DOUBLES(M));
        std::vector<double> cf;
        double* g = gy;
        for (int q = 0; q < nrhs; ++q) {
            fh_status st = run_moments(b, nrhs, q, P, rec.data(), s, M + 1);
            if (st != FH_OK) return st;
            if ((st = terminal_coefficients(M, rec.data(), objective, obj_mode, &J[q], cf)) != FH_OK) return st;
            if ((st = run_onebody(b, nrhs, q, P, g, cf, s)) != FH_OK) return st;
            const int nb = launch_dot_re(g, Z, b->total, nrhs, q, b->d_partial, s);
            launch_reduce_partials(b->d_partial, 1, nb, 1, 1, b->d_small, 0, s);
            FH_HIP(hipGetLastError());
            FH_HIP(hipMemcpyAsync(&dJ_dLambda[q], b->d_small, sizeof(double), hipMemcpyDeviceToHost, s));
            FH_HIP(hipStreamSynchronize(s));
        }
        return FH_OK;
    });
}

int fh_chebyshev_coefficients(double x, double tol, int kmax, double* c_re, double* c_im) {
    if (!std::isfinite(x) || x < 0.0 || !(tol > 0.0) || kmax < 2 || x >= (double)kmax) return -1;
    int k = (int)x + 1;
    while (k <= x || 2.0 * std::fabs(std::cyl_bessel_j((double)k, x)) >= tol) {
        if (++k >= kmax) return -1;
    }
    const int K = k + 1;
    if (K > kmax) return -1;
    static const double pr[4] = {1.0, 0.0, -1.0, 0.0}, pi[4] = {0.0, -1.0, 0.0, 1.0};  // (-i)^j
    for (int j = 0; j < K; ++j) {
        const double J = (j == 0 ? 1.0 : 2.0) * std::cyl_bessel_j((double)j, x);
        if (c_re) c_re[j] = pr[j & 3] * J;
        if (c_im) c_im[j] = pi[j & 3] * J;
    }
    return K;
}

fh_status fh_spectral_radius(const fh_model* m, const fh_basis* b, fh_c64* work, int iters, double* rho,
                             void* stream) {
    return Guard::run([&]() -> fh_status {
        if (!check_model_basis(m, b)) return FH_EINVAL;
        FH_REQUIRE(work && rho && iters >= 1, FH_EINVAL, "fh_spectral_radius: bad argument");
        hipStream_t s = as_stream(stream);
        const int64_t vec = 2 * b->total;
        double* x = reinterpret_cast<double*>(work);
        double* y = x + vec;
        auto norm2 = [&](const double* v, double* out) -> fh_status {
            const int nb = launch_dot_re(v, v, b->total, 1, 0, b->d_partial, s);
            launch_reduce_partials(b->d_partial, 1, nb, 1, 1, b->d_small, 0, s);
            FH_HIP(hipGetLastError());
            FH_HIP(hipMemcpyAsync(out, b->d_small, sizeof(double), hipMemcpyDeviceToHost, s));
            FH_HIP(hipStreamSynchronize(s));
            return FH_OK;
        };
        launch_hash_fill(x, b->total, 0x5eed5eedull, s);
        double nx = 0.0, ny = 0.0, r = 0.0;
        fh_status st = norm2(x, &nx);
        if (st != FH_OK) return st;
        FH_REQUIRE(nx > 0.0, FH_ESTATE, "fh_spectral_radius: empty basis");
        for (int it = 0; it < iters; ++it) {
            StageArgs a = stage_base(m, b);
            a.x = x;
            a.out = y;
            a.mode = kApply;
            if ((st = launch_stage(b, 1, a, 0, s, nullptr)) != FH_OK) return st;
            if ((st = norm2(y, &ny)) != FH_OK) return st;
            r = std::sqrt(ny / nx);
            if (ny == 0.0) break;
            launch_cscale(x, y, b->total, 1.0 / std::sqrt(ny), 0.0, s);
            nx = 1.0;
        }
        *rho = r;
        return FH_OK;
    });
}

fh_status fh_evolve_chebyshev(const fh_model* m, const fh_basis* b, int nrhs, fh_c64* psi, fh_c64* work, double dt,
                              int64_t nsteps, double emin, double emax, double tol, int64_t obs_every,
                              double* moments, int64_t moments_capacity, int flags, fh_timing* timing,
                              void* stream) {
    return Guard::run([&]() -> fh_status {
        const auto t0 = std::chrono::steady_clock::now();
        if (!check_model_basis(m, b)) return FH_EINVAL;
        FH_REQUIRE(!bad_nrhs(nrhs), FH_EINVAL, "nrhs must be 1, 2, 4, 8 or 16");
        FH_REQUIRE(psi && work, FH_EINVAL, "fh_evolve_chebyshev: NULL buffer");
        FH_REQUIRE(nsteps >= 0 && obs_every >= 0, FH_EINVAL, "fh_evolve_chebyshev: negative step count");
        FH_REQUIRE(std::isfinite(dt) && dt >= 0.0, FH_EINVAL, "fh_evolve_chebyshev: dt must be finite and >= 0");
        FH_REQUIRE(std::isfinite(emin) && std::isfinite(emax) && emax > emin, FH_EINVAL,
                   "fh_evolve_chebyshev: need finite emin < emax");
        FH_REQUIRE(tol > 0.0, FH_EINVAL, "fh_evolve_chebyshev: tol must be > 0");
        FH_REQUIRE(!(flags & FH_GRAPH), FH_EINVAL, "fh_evolve_chebyshev: FH_GRAPH is not supported");
        const int M = b->M;
        hipStream_t s = as_stream(stream);
        const double a = 0.5 * (emax + emin), bw = 0.5 * (emax - emin);
        std::vector<double> cre(4096), cim(4096);  // up to 4096 terms: (emax - emin) dt / 2 < ~4000
        const int K = fh_chebyshev_coefficients(bw * dt, tol, (int)cre.size(), cre.data(), cim.data());
        FH_REQUIRE(K >= 2, FH_EUNSUPPORTED, "fh_evolve_chebyshev: (emax - emin) * dt too large for one step");
        const int64_t vec = 2 * b->total * nrhs;
        const long long ncplx = (long long)b->total * nrhs;
        double* P = reinterpret_cast<double*>(psi);
        double* A = reinterpret_cast<double*>(work);
        double* B = A + vec;
        double* h = A + 2 * vec;
        double* acc = A + 3 * vec;
        const int64_t nrec = obs_every > 0 ? nsteps / obs_every + 1 : 0;
        const int64_t per = (int64_t)FH_MOMENT_DOUBLES(M) * nrhs;
        if (nrec > 0) {
            FH_REQUIRE(moments != nullptr, FH_EINVAL, "fh_evolve_chebyshev: moments buffer is NULL");
            FH_REQUIRE(moments_capacity >= nrec * per, FH_ENOMEM, "fh_evolve_chebyshev: moments buffer too small");
        }
        StageTimer tm;
        fh_status st = tm.init((flags & FH_TIMING) != 0, s);
        if (st != FH_OK) return st;
        StageTimer* tmp = (flags & FH_TIMING) ? &tm : nullptr;
        auto norm2 = [&](double* out) -> fh_status {
            const int nb = launch_dot_re(P, P, ncplx, 1, 0, b->d_partial, s);
            launch_reduce_partials(b->d_partial, 1, nb, 1, 1, b->d_small, 0, s);
            FH_HIP(hipGetLastError());
            FH_HIP(hipMemcpyAsync(out, b->d_small, sizeof(double), hipMemcpyDeviceToHost, s));
            FH_HIP(hipStreamSynchronize(s));
            return FH_OK;
        };
        auto apply = [&](const double* x) -> fh_status {
            StageArgs sa = stage_base(m, b);
            sa.x = x;
            sa.out = h;
            sa.mode = kApply;
            return launch_stage(b, nrhs, sa, flags, s, tmp);
        };
        auto record = [&](int64_t r) -> fh_status {
            for (int q = 0; q < nrhs; ++q) {
                fh_status e = run_moments(b, nrhs, q, P, moments + r * per + (int64_t)q * FH_MOMENT_DOUBLES(M), s,
                                          M + 1);
                if (e != FH_OK) return e;
            }
            return FH_OK;
        };
        double n0 = 0.0, n1 = 0.0;
        if ((st = norm2(&n0)) != FH_OK) return st;
        int64_t r = 0;
        if (nrec > 0 && (st = record(r++)) != FH_OK) return st;
        const double ph_re = std::cos(a * dt), ph_im = -std::sin(a * dt);
        for (int64_t step = 1; step <= nsteps; ++step) {
            // T_1 psi = (H - a) psi / b;  acc = c_0 psi + c_1 T_1 psi
            if ((st = apply(P)) != FH_OK) return st;
            launch_cheb_term(h, P, nullptr, B, acc, ncplx, 1.0 / bw, -a / bw, 0.0, cre[1], cim[1], 1, cre[0], cim[0], s);
            const double* prev = P;
            double* cur = B;
            for (int k = 2; k < K; ++k) {
                // T_k = 2 (H - a)/b T_{k-1} - T_{k-2}, written over T_{k-2} (never over psi)
                if ((st = apply(cur)) != FH_OK) return st;
                double* dest = prev == P ? A : const_cast<double*>(prev);
                launch_cheb_term(h, cur, prev, dest, acc, ncplx, 2.0 / bw, -2.0 * a / bw, -1.0, cre[k], cim[k], 0, 0.0,
                                 0.0, s);
                prev = cur;
                cur = dest;
            }
            launch_cscale(P, acc, ncplx, ph_re, ph_im, s);  // psi = exp(-i a dt) acc
            FH_HIP(hipGetLastError());
            if (obs_every > 0 && step % obs_every == 0 && (st = record(r++)) != FH_OK) return st;
        }
        st = tm.flush();
        if (st != FH_OK) return st;
        if ((st = norm2(&n1)) != FH_OK) return st;
        // exp(-i H t) keeps the norm; a series that left [-1, 1] grows without bound
        FH_REQUIRE(std::isfinite(n1) && std::fabs(n1 - n0) <= 1e-8 * std::max(n0, 1e-300), FH_ESTATE,
                   "fh_evolve_chebyshev: norm not conserved; the spectrum of H is not inside [emin, emax]");
        if (timing) {
            timing->stage_ms = tm.ms;
            timing->stage_launches = tm.launches;
            timing->wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        }
        return FH_OK;
    });
}

fh_status fh_coherent_vjp(const fh_basis* b, int nrhs, const fh_c64* alpha, const fh_c64* lambda0, double* d_re,
                          double* d_im, void* stream) {
    return Guard::run([&]() -> fh_status {
        FH_REQUIRE(b && alpha && lambda0 && d_re && d_im, FH_EINVAL, "fh_coherent_vjp: NULL argument");
        FH_REQUIRE(!bad_nrhs(nrhs), FH_EINVAL, "nrhs must be 1, 2, 4, 8 or 16");
        const int M = b->M, Wd = b->Nmax + 1, nt = (int)b->tiles.size();
        hipStream_t s = as_stream(stream);
        for (int q = 0; q < nrhs; ++q) {
            std::vector<double> tabs((size_t)2 * M * Wd * 2);
            double* tab = tabs.data();
            double* tabd = tab + (size_t)M * Wd * 2;
            for (int mm = 0; mm < M; ++mm) {
                const std::complex<double> a(alpha[q * M + mm].re, alpha[q * M + mm].im);
                std::complex<double> t = std::exp(-0.5 * std::norm(a));
                std::complex<double> prev = 0.0;
                for (int n = 0; n < Wd; ++n) {
                    if (n > 0) {
                        prev = t;
                        t = t * a / std::sqrt((double)n);
                    }
                    // n a^(n-1)/sqrt(n!) e^{-|a|^2/2} = sqrt(n) * (a^(n-1)/sqrt((n-1)!) e^{-|a|^2/2})
                    const std::complex<double> d = n > 0 ? std::sqrt((double)n) * prev : 0.0;
                    tab[((size_t)mm * Wd + n) * 2] = t.real();
                    tab[((size_t)mm * Wd + n) * 2 + 1] = t.imag();
                    tabd[((size_t)mm * Wd + n) * 2] = d.real();
                    tabd[((size_t)mm * Wd + n) * 2 + 1] = d.imag();
                }
            }
            FH_HIP(hipMemcpyAsync(b->d_small, tabs.data(), sizeof(double) * tabs.size(), hipMemcpyHostToDevice, s));
            std::vector<double> S(2 * (M + 1), 0.0);
            if (nt > 0) {
                VjpArgs a{};
                a.g = reinterpret_cast<const double*>(lambda0);
                a.nrhs = nrhs;
                a.rhs = q;
                a.T = b->d_T;
                a.Tn = b->Tn;
                a.Rdim = b->Rdim;
                a.tiles = b->d_tiles;
                a.ntiles = nt;
                a.secs = b->d_secs;
                a.tab = b->d_small;
                a.tabd = b->d_small + (size_t)M * Wd * 2;
                a.Nmax = b->Nmax;
                a.partial = b->d_partial;
                const size_t lds = sizeof(int) * (size_t)lds_sqrt_offset(b->Tn) + sizeof(double) * 4 * 2 * (M + 1);
                const int G = std::min(nt, b->grid_cap);
                b->ks->vjp(a, G, lds, s);
                FH_HIP(hipGetLastError());
                double* red = b->d_small + tabs.size();
                launch_reduce_partials(b->d_partial, 1, G, 2 * (kMaxM + 1), 2 * (M + 1), red, 0, s);
                FH_HIP(hipGetLastError());
                FH_HIP(hipMemcpyAsync(S.data(), red, sizeof(double) * S.size(), hipMemcpyDeviceToHost, s));
                FH_HIP(hipStreamSynchronize(s));
            }
            const double reS0 = S[0];
            for (int k = 0; k < M; ++k) {
                const double sr = S[2 * (k + 1)], si = S[2 * (k + 1) + 1];
                d_re[q * M + k] = sr - alpha[q * M + k].re * reS0;
                d_im[q * M + k] = -si - alpha[q * M + k].im * reS0;
            }
        }
        return FH_OK;
    });
}

}  // extern "C"

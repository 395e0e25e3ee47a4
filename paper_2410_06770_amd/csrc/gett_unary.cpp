// gett_unary.cpp -- host side of the unary operations (transpose, reduction,
// trace): argument checks, canonical form, offset tables, launches.
//
// The call is C[PERM(rest)] <- alpha * sum_{summed coordinates} A + beta * C_in,
// where `rest` are A's modes that are neither summed (SUMA) nor in a trace
// pair (TRA[t] with TRB[t], one coordinate walking both modes).  A trace
// pair is a single summed mode whose increment is the sum of the pair's
// increments; a transpose sums nothing.  The planner drops extent-1 modes,
// merges modes that continue each other, and picks the kernel whose lanes
// run along A's cheapest mode: an output mode (tiled kernel) or a summed one
// (lanes-along-R kernel).
#include <algorithm>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "gett.h"
#include "gett_internal.h"
#include "gett_unary.h"

namespace gett {

namespace {

constexpr int64_t kMaxRankU = 64;

int64_t iabs(int64_t x) { return x < 0 ? -x : x; }

bool span_fits(int64_t rank, const int64_t *ext, const int64_t *inc) {
    __int128 total = 0;
    for (int64_t i = 0; i < rank; ++i) {
        if (ext[i] <= 1) continue;
        const __int128 a = inc[i] < 0 ? -(__int128)inc[i] : (__int128)inc[i];
        total += a * (__int128)(ext[i] - 1);
        if (total > INT64_MAX) return false;
    }
    return true;
}

bool count_fits(int64_t rank, const int64_t *ext, int64_t *n) {
    __int128 p = 1;
    for (int64_t i = 0; i < rank; ++i) {
        p *= ext[i];
        if (p > INT64_MAX) return false;
    }
    *n = (int64_t)p;
    return true;
}

struct UArgs {
    int64_t ranka;
    const int64_t *exta, *inca;
    int64_t nsum;
    const int64_t *suma;
    int64_t ntr;
    const int64_t *tra, *trb, *perm, *incc;
};

// INFO in the argument order ALPHA, RANKA, EXTA, INCA, A, NSUM, SUMA, NTR,
// TRA, TRB, PERM, INCC, BETA, C.
int validate_unary(const UArgs &u, const void *A, const void *C) {
    if (u.ranka < 0 || u.ranka > kMaxRankU) return -2;
    if (u.ranka > 0 && !u.exta) return -3;
    for (int64_t i = 0; i < u.ranka; ++i)
        if (u.exta[i] < 0) return -3;
    int64_t na = 0;
    if (!count_fits(u.ranka, u.exta, &na)) return -3;
    if (u.ranka > 0 && (!u.inca || !span_fits(u.ranka, u.exta, u.inca))) return -4;
    if (na > 0 && !A) return -5;
    if (u.nsum < 0 || u.nsum > u.ranka) return -6;
    if (u.nsum > 0 && !u.suma) return -7;
    bool used[kMaxRankU] = {false};
    for (int64_t k = 0; k < u.nsum; ++k) {
        const int64_t x = u.suma[k];
        if (x < 0 || x >= u.ranka || used[x]) return -7;
        used[x] = true;
    }
    if (u.ntr < 0 || u.nsum + 2 * u.ntr > u.ranka) return -8;
    if (u.ntr > 0 && !u.tra) return -9;
    for (int64_t t = 0; t < u.ntr; ++t) {
        const int64_t x = u.tra[t];
        if (x < 0 || x >= u.ranka || used[x]) return -9;
        used[x] = true;
    }
    if (u.ntr > 0 && !u.trb) return -10;
    for (int64_t t = 0; t < u.ntr; ++t) {
        const int64_t y = u.trb[t];
        if (y < 0 || y >= u.ranka || used[y]) return -10;
        used[y] = true;
        if (u.exta[y] != u.exta[u.tra[t]]) return -10;
    }
    const int64_t rc = u.ranka - u.nsum - 2 * u.ntr;
    if (rc > 0 && !u.perm) return -11;
    bool seen[kMaxRankU] = {false};
    for (int64_t p = 0; p < rc; ++p) {
        const int64_t q = u.perm[p];
        if (q < 0 || q >= rc || seen[q]) return -11;
        seen[q] = true;
    }
    int64_t extc[kMaxRankU];
    int64_t p = 0;
    for (int64_t i = 0; i < u.ranka; ++i)
        if (!used[i]) extc[u.perm[p++]] = u.exta[i];
    if (rc > 0 && !u.incc) return -12;
    for (int64_t q = 0; q < rc; ++q)
        if (u.incc[q] == 0 && extc[q] > 1) return -12;
    if (rc > 0 && !span_fits(rc, extc, u.incc)) return -12;
    int64_t nc = 0;
    if (!count_fits(rc, extc, &nc)) return -12;
    if (nc > 0 && !C) return -14;
    return 0;
}

struct OMode {
    int64_t ext, ia, ic;
};
struct RMode {
    int64_t ext, ia;
};

// Canonical form: output modes (extent-1 dropped, continuing modes merged)
// and summed modes (likewise, ordered by |increment in A|).
struct UCanon {
    bool no_outputs = false, empty_sum = false;
    std::vector<OMode> o;
    std::vector<RMode> r;
};

UCanon canonical_unary(const UArgs &u) {
    UCanon c;
    bool summed[kMaxRankU] = {false};
    for (int64_t k = 0; k < u.nsum; ++k) summed[u.suma[k]] = true;
    for (int64_t t = 0; t < u.ntr; ++t) summed[u.tra[t]] = summed[u.trb[t]] = true;
    int64_t p = 0;
    for (int64_t i = 0; i < u.ranka; ++i)
        if (!summed[i]) {
            const int64_t q = u.perm[p++];
            if (u.exta[i] == 0) c.no_outputs = true;
            c.o.push_back({u.exta[i], u.inca[i], u.incc[q]});
        }
    for (int64_t k = 0; k < u.nsum; ++k) c.r.push_back({u.exta[u.suma[k]], u.inca[u.suma[k]]});
    for (int64_t t = 0; t < u.ntr; ++t)
        c.r.push_back({u.exta[u.tra[t]], u.inca[u.tra[t]] + u.inca[u.trb[t]]});
    for (const auto &x : c.r)
        if (x.ext == 0) c.empty_sum = true;
    c.o.erase(std::remove_if(c.o.begin(), c.o.end(), [](const OMode &x) { return x.ext == 1; }),
              c.o.end());
    c.r.erase(std::remove_if(c.r.begin(), c.r.end(), [](const RMode &x) { return x.ext == 1; }),
              c.r.end());
    // merge mode y into x when y continues x (in A and C for outputs, in A
    // for summed modes): a relabelling of the same positions
    for (bool changed = true; changed;) {
        changed = false;
        for (size_t x = 0; x < c.o.size() && !changed; ++x)
            for (size_t y = 0; y < c.o.size() && !changed; ++y)
                if (x != y && (__int128)c.o[y].ia == (__int128)c.o[x].ia * c.o[x].ext &&
                    (__int128)c.o[y].ic == (__int128)c.o[x].ic * c.o[x].ext) {
                    c.o[x].ext *= c.o[y].ext;
                    c.o.erase(c.o.begin() + y);
                    changed = true;
                }
    }
    for (bool changed = true; changed;) {
        changed = false;
        for (size_t x = 0; x < c.r.size() && !changed; ++x)
            for (size_t y = 0; y < c.r.size() && !changed; ++y)
                if (x != y && (__int128)c.r[y].ia == (__int128)c.r[x].ia * c.r[x].ext) {
                    c.r[x].ext *= c.r[y].ext;
                    c.r.erase(c.r.begin() + y);
                    changed = true;
                }
    }
    std::stable_sort(c.r.begin(), c.r.end(),
                     [](const RMode &a, const RMode &b) { return iabs(a.ia) < iabs(b.ia); });
    return c;
}

// A plan: the kernel choice, the O1/O2 split and the O3 and R tables in
// device memory (cached per signature).
struct UPlan {
    bool lanes_r = false, trans = false;
    bool r_affine = false;       // R is a single mode
    int64_t r_inc = 0;
    OMode o1{1, 0, 0}, o2{1, 0, 0};
    int64_t n3 = 1, nR = 1;
    int32_t g = 64;
    int64_t *d_tab = nullptr;   // offA3, offC3 [n3]; offR [nR]
    ~UPlan() {
        if (d_tab) (void)hipFree(d_tab);
    }
};

std::mutex g_umu;
std::map<std::string, std::unique_ptr<UPlan>> g_uplans;

std::string unary_key(const UArgs &u, int prec, int dev) {
    std::vector<int64_t> v{prec, dev, u.ranka};
    for (int64_t i = 0; i < u.ranka; ++i) {
        v.push_back(u.exta[i]);
        v.push_back(u.inca[i]);
    }
    v.push_back(u.nsum);
    for (int64_t k = 0; k < u.nsum; ++k) v.push_back(u.suma[k]);
    v.push_back(u.ntr);
    for (int64_t t = 0; t < u.ntr; ++t) {
        v.push_back(u.tra[t]);
        v.push_back(u.trb[t]);
    }
    const int64_t rc = u.ranka - u.nsum - 2 * u.ntr;
    for (int64_t q = 0; q < rc; ++q) {
        v.push_back(u.perm[q]);
        v.push_back(u.incc[q]);
    }
    return std::string(reinterpret_cast<const char *>(v.data()), v.size() * sizeof(int64_t));
}

int build_plan(const UCanon &c, UPlan &pl) {
    std::vector<OMode> o = c.o;
    int64_t mina_o = INT64_MAX;
    for (const auto &x : o) mina_o = std::min(mina_o, iabs(x.ia));
    const int64_t mina_r = c.r.empty() ? INT64_MAX : iabs(c.r[0].ia);
    pl.lanes_r = !c.r.empty() && mina_r < mina_o;
    auto take = [&](bool by_a) {
        if (o.empty()) return OMode{1, 0, 0};
        size_t b = 0;
        for (size_t i = 1; i < o.size(); ++i)
            if ((by_a ? iabs(o[i].ia) < iabs(o[b].ia) : iabs(o[i].ic) < iabs(o[b].ic))) b = i;
        const OMode m = o[b];
        o.erase(o.begin() + b);
        return m;
    };
    if (pl.lanes_r) {
        // outputs numbered along C's cheapest modes (neighbouring output
        // groups of a wave store to neighbouring addresses)
        pl.o1 = take(false);
        pl.o2 = take(false);
    } else {
        pl.o1 = take(true);
        int64_t minc = iabs(pl.o1.ic);
        for (const auto &x : o) minc = std::min(minc, iabs(x.ic));
        pl.trans = !o.empty() && minc < iabs(pl.o1.ic);
        pl.o2 = take(false);
    }
    // O3 and R tables (odometer, first mode fastest)
    pl.n3 = 1;
    for (const auto &x : o) pl.n3 *= x.ext;
    pl.nR = 1;
    for (const auto &x : c.r) pl.nR *= x.ext;
    if (pl.n3 > ((int64_t)1 << 31) || pl.nR > ((int64_t)1 << 31)) return GETT_ERR_INTERNAL;
    std::vector<int64_t> h(2 * pl.n3 + pl.nR);
    for (int64_t i = 0; i < pl.n3; ++i) {
        int64_t r = i, oa = 0, oc = 0;
        for (const auto &x : o) {
            const int64_t k = r % x.ext;
            r /= x.ext;
            oa += k * x.ia;
            oc += k * x.ic;
        }
        h[i] = oa;
        h[pl.n3 + i] = oc;
    }
    for (int64_t i = 0; i < pl.nR; ++i) {
        int64_t r = i, oa = 0;
        for (const auto &x : c.r) {
            oa += (r % x.ext) * x.ia;
            r /= x.ext;
        }
        h[2 * pl.n3 + i] = oa;
    }
    int g = 1;
    while (g < 64 && g < pl.nR) g <<= 1;
    pl.g = g;
    pl.r_affine = c.r.size() == 1;
    pl.r_inc = pl.r_affine ? c.r[0].ia : 0;
    const size_t bytes = h.size() * sizeof(int64_t);
    if (hipMalloc(&pl.d_tab, bytes) != hipSuccess) return GETT_ERR_ALLOC;
    if (hipMemcpy(pl.d_tab, h.data(), bytes, hipMemcpyHostToDevice) != hipSuccess)
        return GETT_ERR_HIP;
    return 0;
}

int run_unary(int prec, const double *alpha, const UArgs &u, const void *A, const double *beta,
              void *C) {
    const int info = validate_unary(u, A, C);
    if (info) return info;
    const UCanon c = canonical_unary(u);
    if (c.no_outputs) return 0;
    int dev = 0;
    int rc = current_device_checked(&dev);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(gett_get_stream());
    if (c.empty_sum) {
        // nothing summed: C <- beta * C_in on every output
        if (beta[0] == 1.0 && beta[1] == 0.0) return 0;
        ScaleModes sm{};
        sm.total = 1;
        for (const auto &x : c.o) {
            if (sm.n >= kScaleModes) return GETT_ERR_INTERNAL;
            sm.ext[sm.n] = x.ext;
            sm.inc[sm.n] = x.ic;
            ++sm.n;
            sm.total *= x.ext;
        }
        return launch_scale_c(prec, C, sm, beta, s);
    }
    const std::string key = unary_key(u, prec, dev);
    UPlan *pl = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_umu);
        auto it = g_uplans.find(key);
        if (it != g_uplans.end()) pl = it->second.get();
    }
    if (!pl) {
        auto np = std::make_unique<UPlan>();
        rc = build_plan(c, *np);
        if (rc) return rc;
        std::lock_guard<std::mutex> lk(g_umu);
        auto &slot = g_uplans[key];
        if (!slot) slot = std::move(np);
        pl = slot.get();
    }
    UnaryParams p{};
    p.A = A;
    p.C = C;
    p.e1 = pl->o1.ext;
    p.e2 = pl->o2.ext;
    p.ia1 = pl->o1.ia;
    p.ia2 = pl->o2.ia;
    p.ic1 = pl->o1.ic;
    p.ic2 = pl->o2.ic;
    p.offA3 = pl->d_tab;
    p.offC3 = pl->d_tab + pl->n3;
    p.n3 = pl->n3;
    p.offR = pl->d_tab + 2 * pl->n3;
    p.nR = pl->nR;
    p.nO = p.e1 * p.e2 * p.n3;
    p.g = pl->g;
    p.trans = pl->trans ? 1 : 0;
    p.rAffine = pl->r_affine ? 1 : 0;
    p.rInc = pl->r_inc;
    p.tiles1 = (int32_t)((p.e1 + 63) / 64);
    p.tiles2 = (int32_t)((p.e2 + 63) / 64);
    for (int i = 0; i < 2; ++i) {
        p.alpha[i] = alpha[i];
        p.beta[i] = beta[i];
    }
    // Slices of the summed positions when the outputs alone cannot fill the
    // chip: FP64 partials, added in slice order by the finishing kernel.
    int64_t S = 1;
    if (pl->lanes_r) {
        const int64_t groups = (p.nO + (64 / p.g) - 1) / (64 / p.g);   // wave rounds
        if (groups < 4096 && p.nR > 8 * (int64_t)p.g)
            S = std::min<int64_t>((8192 + groups - 1) / groups, p.nR / (4 * (int64_t)p.g));
    } else {
        const int64_t blocks = (int64_t)p.tiles1 * p.tiles2 * p.n3;
        // a workgroup of the one-output-row variant walks 64 positions a round
        const int64_t minPer = p.e2 == 1 ? 256 : 32;
        if (blocks < 1024 && p.nR > 2 * minPer)
            S = std::min<int64_t>((2048 + blocks - 1) / blocks, p.nR / minPer);
    }
    if (S < 1) S = 1;
    int64_t per = (p.nR + S - 1) / S;
    S = (p.nR + per - 1) / per;
    p.rPer = per;
    p.S = (int32_t)S;
    void *ws = nullptr;
    if (S > 1) {
        const int64_t bytes = S * p.nO * (prec >= 4 ? 2 : 1) * (int64_t)sizeof(double);
        if (work_alloc(&ws, (size_t)bytes, s)) {   // no workspace: one slice
            p.S = 1;
            p.rPer = p.nR;
        } else {
            p.ws = static_cast<double *>(ws);
        }
    }
    rc = pl->lanes_r ? launch_unary_lanes_r(prec, p, s) : launch_unary_tiled(prec, p, s);
    if (!rc && p.S > 1) rc = launch_unary_finish(prec, p, s);
    if (ws && work_free(ws, s) && !rc) rc = GETT_ERR_HIP;
    return rc;
}

}  // namespace

void unary_release() {
    std::lock_guard<std::mutex> lk(g_umu);
    g_uplans.clear();
}

}  // namespace gett

using namespace gett;

#define GETT_UNARY_ARGS UArgs{ranka, exta, inca, nsum, suma, ntr, tra, trb, perm, incc}

extern "C" {

int dgett_unary(double alpha, int64_t ranka, const int64_t *exta, const int64_t *inca,
                const double *A, int64_t nsum, const int64_t *suma, int64_t ntr,
                const int64_t *tra, const int64_t *trb, const int64_t *perm, const int64_t *incc,
                double beta, double *C) {
    const double al[2] = {alpha, 0.0}, be[2] = {beta, 0.0};
    return run_unary(0, al, GETT_UNARY_ARGS, A, be, C);
}

int sgett_unary(float alpha, int64_t ranka, const int64_t *exta, const int64_t *inca,
                const float *A, int64_t nsum, const int64_t *suma, int64_t ntr,
                const int64_t *tra, const int64_t *trb, const int64_t *perm, const int64_t *incc,
                float beta, float *C) {
    const double al[2] = {alpha, 0.0}, be[2] = {beta, 0.0};
    return run_unary(1, al, GETT_UNARY_ARGS, A, be, C);
}

int zgett_unary(const double *alpha, int64_t ranka, const int64_t *exta, const int64_t *inca,
                const void *A, int64_t nsum, const int64_t *suma, int64_t ntr,
                const int64_t *tra, const int64_t *trb, const int64_t *perm, const int64_t *incc,
                const double *beta, void *C) {
    if (!alpha) return -1;
    if (!beta) return -13;
    return run_unary(4, alpha, GETT_UNARY_ARGS, A, beta, C);
}

int cgett_unary(const float *alpha, int64_t ranka, const int64_t *exta, const int64_t *inca,
                const void *A, int64_t nsum, const int64_t *suma, int64_t ntr,
                const int64_t *tra, const int64_t *trb, const int64_t *perm, const int64_t *incc,
                const float *beta, void *C) {
    if (!alpha) return -1;
    if (!beta) return -13;
    const double al[2] = {alpha[0], alpha[1]}, be[2] = {beta[0], beta[1]};
    return run_unary(5, al, GETT_UNARY_ARGS, A, be, C);
}

}  // extern "C"

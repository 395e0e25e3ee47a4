// gett_plan.cpp -- argument checks, M/N/K grouping and offset tables (host only,
// no HIP calls: the CPU tests load the library and exercise this file).
//
// Section 6 of the paper first rewrites the arguments into a "manageable
// format": the free extents in output order with their owning tensor and
// increments, the contracted extents with the increments of A and B, and the
// increments of C.  The planner builds the same description and then
// regroups it for a matrix-core GEMM:
//   M = free modes of A, N = free modes of B, K = contracted pairs,
// each mode carrying the increments of the two tensors that see it.  It
// drops extent-1 modes, merges modes that are jointly contiguous in both
// tensors of their group, and orders the modes of each group so that the
// first (fastest) mode is the cheapest direction in memory.  Swapping A and B
// (Section 7, Commutativity: the same contraction with the PERM entries of
// the two free lists exchanged) puts C's fastest mode into N, which is the
// lane axis of the MFMA result.
#include "gett_plan.h"

#include <algorithm>
#include <cmath>
#include <cstring>

#include "gett.h"

namespace gett {

static const int64_t kMaxRank = 64;

static int64_t iabs(int64_t x) { return x < 0 ? -x : x; }

static bool mul_ok(int64_t a, int64_t b, int64_t *r) {
    __int128 p = (__int128)a * (__int128)b;
    if (p > INT64_MAX || p < INT64_MIN) return false;
    *r = (int64_t)p;
    return true;
}

// sum |inc| * (ext - 1) fits in int64
static bool span_ok(int64_t rank, const int64_t *ext, const int64_t *inc) {
    __int128 total = 0;
    for (int64_t i = 0; i < rank; ++i) {
        if (ext[i] <= 1) continue;
        __int128 a = inc[i] < 0 ? -(__int128)inc[i] : (__int128)inc[i];
        total += a * (__int128)(ext[i] - 1);
        if (total > INT64_MAX) return false;
    }
    return true;
}

static bool count_ok(int64_t rank, const int64_t *ext, int64_t *n) {
    int64_t p = 1;
    for (int64_t i = 0; i < rank; ++i)
        if (!mul_ok(p, ext[i], &p)) return false;
    *n = p;
    return true;
}

int validate(const Args &a, const void *A, const void *B, const void *C) {
    int64_t na = 0, nb = 0;
    if (a.ranka < 0 || a.ranka > kMaxRank) return -1;
    if (a.ranka > 0 && !a.exta) return -2;
    for (int64_t i = 0; i < a.ranka; ++i)
        if (a.exta[i] < 0) return -2;
    if (a.ranka > 0 && !a.inca) return -3;
    if (a.ranka > 0 && !span_ok(a.ranka, a.exta, a.inca)) return -3;
    if (!count_ok(a.ranka, a.exta, &na)) return -2;
    if (na > 0 && !A) return -4;

    if (a.rankb < 0 || a.rankb > kMaxRank) return -5;
    if (a.rankb > 0 && !a.extb) return -6;
    for (int64_t i = 0; i < a.rankb; ++i)
        if (a.extb[i] < 0) return -6;
    if (a.rankb > 0 && !a.incb) return -7;
    if (a.rankb > 0 && !span_ok(a.rankb, a.extb, a.incb)) return -7;
    if (!count_ok(a.rankb, a.extb, &nb)) return -6;
    if (nb > 0 && !B) return -8;

    if (a.conts < 0 || a.conts > a.ranka || a.conts > a.rankb) return -9;
    if (a.conts > 0 && !a.conta) return -10;
    bool usedA[kMaxRank] = {false}, usedB[kMaxRank] = {false};
    for (int64_t k = 0; k < a.conts; ++k) {
        const int64_t x = a.conta[k];
        if (x < 0 || x >= a.ranka || usedA[x]) return -10;
        usedA[x] = true;
    }
    if (a.conts > 0 && !a.contb) return -11;
    for (int64_t k = 0; k < a.conts; ++k) {
        const int64_t y = a.contb[k];
        if (y < 0 || y >= a.rankb || usedB[y]) return -11;
        usedB[y] = true;
        if (a.exta[a.conta[k]] != a.extb[y]) return -11;   // Section 2.2: equal extents
    }
    // Hadamard pairs: modes of A and B not contracted, each used once, equal
    // extents.
    if (a.hads < 0 || a.conts + a.hads > a.ranka || a.conts + a.hads > a.rankb) return kInfoHads;
    if (a.hads > 0 && !a.hada) return kInfoHada;
    bool hadA[kMaxRank] = {false}, hadB[kMaxRank] = {false};
    for (int64_t h = 0; h < a.hads; ++h) {
        const int64_t x = a.hada[h];
        if (x < 0 || x >= a.ranka || usedA[x] || hadA[x]) return kInfoHada;
        hadA[x] = true;
    }
    if (a.hads > 0 && !a.hadb) return kInfoHadb;
    for (int64_t h = 0; h < a.hads; ++h) {
        const int64_t y = a.hadb[h];
        if (y < 0 || y >= a.rankb || usedB[y] || hadB[y]) return kInfoHadb;
        hadB[y] = true;
        if (a.exta[a.hada[h]] != a.extb[y]) return kInfoHadb;
    }
    const int64_t rc = out_rank(a);
    if (rc > 0 && !a.perm) return -12;
    bool seen[2 * kMaxRank] = {false};
    for (int64_t p = 0; p < rc; ++p) {
        const int64_t q = a.perm[p];
        if (q < 0 || q >= rc || seen[q]) return -12;
        seen[q] = true;
    }
    int64_t extc[2 * kMaxRank];
    int64_t p = 0;
    for (int64_t i = 0; i < a.ranka; ++i)
        if (!usedA[i] && !hadA[i]) extc[a.perm[p++]] = a.exta[i];
    for (int64_t j = 0; j < a.rankb; ++j)
        if (!usedB[j] && !hadB[j]) extc[a.perm[p++]] = a.extb[j];
    for (int64_t h = 0; h < a.hads; ++h) extc[a.perm[p++]] = a.exta[a.hada[h]];
    if (rc > 0 && !a.incc) return -13;
    for (int64_t q = 0; q < rc; ++q)
        if (a.incc[q] == 0 && extc[q] > 1) return -13;
    if (rc > 0 && !span_ok(rc, extc, a.incc)) return -13;
    int64_t nc = 0;
    if (!count_ok(rc, extc, &nc)) return -13;
    if (nc > 0 && !C) return -14;
    return 0;
}

// Raw groups straight from the arguments (Section 6 preprocessing, regrouped).
static void raw_groups(const Args &a, std::vector<GMode> &m, std::vector<GMode> &n,
                       std::vector<GMode> &k, std::vector<HMode> *hg = nullptr) {
    bool contA[kMaxRank] = {false}, contB[kMaxRank] = {false};
    for (int64_t x = 0; x < a.conts; ++x) {
        contA[a.conta[x]] = true;
        contB[a.contb[x]] = true;
    }
    for (int64_t h = 0; h < a.hads; ++h) {   // Hadamard modes are neither free nor summed
        contA[a.hada[h]] = true;
        contB[a.hadb[h]] = true;
    }
    int64_t p = 0;
    for (int64_t i = 0; i < a.ranka; ++i)
        if (!contA[i]) {
            m.push_back({a.exta[i], a.inca[i], a.incc[a.perm[p]]});
            ++p;
        }
    for (int64_t j = 0; j < a.rankb; ++j)
        if (!contB[j]) {
            n.push_back({a.extb[j], a.incb[j], a.incc[a.perm[p]]});
            ++p;
        }
    for (int64_t x = 0; x < a.conts; ++x)
        k.push_back({a.exta[a.conta[x]], a.inca[a.conta[x]], a.incb[a.contb[x]]});
    if (hg)
        for (int64_t h = 0; h < a.hads; ++h) {
            hg->push_back({a.exta[a.hada[h]], a.inca[a.hada[h]], a.incb[a.hadb[h]],
                           a.incc[a.perm[p]]});
            ++p;
        }
}

static int64_t group_size(const std::vector<GMode> &g) {
    int64_t s = 1;
    for (const auto &x : g) s *= x.ext;
    return s;
}

// Merge mode b into mode a when b continues a in both tensors of the group.
static void merge_group(std::vector<GMode> &g) {
    bool changed = true;
    while (changed) {
        changed = false;
        for (size_t x = 0; x < g.size() && !changed; ++x)
            for (size_t y = 0; y < g.size() && !changed; ++y) {
                if (x == y) continue;
                const __int128 e = g[x].ext;
                if ((__int128)g[y].i0 == (__int128)g[x].i0 * e &&
                    (__int128)g[y].i1 == (__int128)g[x].i1 * e) {
                    g[x].ext *= g[y].ext;
                    g.erase(g.begin() + y);
                    changed = true;
                }
            }
    }
}

static void sort_by(std::vector<GMode> &g, int slot) {
    std::stable_sort(g.begin(), g.end(), [slot](const GMode &u, const GMode &v) {
        const int64_t a0 = iabs(slot ? u.i1 : u.i0), b0 = iabs(slot ? v.i1 : v.i0);
        if (a0 != b0) return a0 < b0;
        return iabs(slot ? u.i0 : u.i1) < iabs(slot ? v.i0 : v.i1);
    });
}

static int64_t min_abs(const std::vector<GMode> &g, int slot) {
    int64_t best = INT64_MAX;
    for (const auto &x : g) best = std::min(best, iabs(slot ? x.i1 : x.i0));
    return best;
}

Canon canonicalise(const Args &a, int order, int bn) {
    Canon c;
    std::vector<GMode> m, n, k;
    std::vector<HMode> h;
    raw_groups(a, m, n, k, &h);
    for (auto *g : {&m, &n, &k})
        for (const auto &x : *g)
            if (x.ext == 0) c.empty = true;
    for (const auto &x : h)
        if (x.ext == 0) c.empty = true;
    h.erase(std::remove_if(h.begin(), h.end(), [](const HMode &x) { return x.ext == 1; }),
            h.end());
    auto drop1 = [](std::vector<GMode> &g) {
        g.erase(std::remove_if(g.begin(), g.end(), [](const GMode &x) { return x.ext == 1; }),
                g.end());
    };
    drop1(m);
    drop1(n);
    drop1(k);

    // Put C's fastest free mode into N (the MFMA result's lane axis).
    int64_t cm = min_abs(m, 1), cn = min_abs(n, 1);
    if (!m.empty() && (n.empty() || cm < cn)) {
        c.swapped = true;
        std::swap(m, n);
        for (auto &x : k) std::swap(x.i0, x.i1);
        for (auto &x : h) std::swap(x.ia, x.ib);
    }
    merge_group(m);
    merge_group(n);
    merge_group(k);

    sort_by(m, 0);
    if (order == 1) sort_by(n, 1);
    else sort_by(n, 0);

    // K: read along K by the operand whose smallest stride is contracted.
    const bool aPrefK = !k.empty() && (m.empty() || min_abs(k, 0) < min_abs(m, 0));
    const bool bPrefK = !k.empty() && (n.empty() || min_abs(k, 1) < min_abs(n, 0));
    sort_by(k, aPrefK ? 0 : (bPrefK ? 1 : 0));

    c.aFastK = !k.empty() && (m.empty() || iabs(k[0].i0) < iabs(m[0].i0));
    c.bFastK = !k.empty() && (n.empty() || iabs(k[0].i1) < iabs(n[0].i0));

    // Orders 2 and 3 box the N tile when B's fastest N mode x is not C's
    // fastest N mode y: a tile of Y positions of y times X of x, y first, so
    // the epilogue's lanes run along y while B's loader runs along x.  Order
    // 2 favours the loads (Y = 4), order 3 the stores (Y = 16).
    if ((order == 2 || order == 3) && !c.bFastK && n.size() >= 2 && bn > 0) {
        size_t yi = 0;
        for (size_t i = 1; i < n.size(); ++i)
            if (iabs(n[i].i1) < iabs(n[yi].i1)) yi = i;
        if (yi != 0 && iabs(n[yi].i1) < iabs(n[0].i1)) {
            const int cand2[3] = {4, 8, 2}, cand3[3] = {16, 8, 32};
            const int *cand = order == 2 ? cand2 : cand3;
            for (int ci = 0; ci < 3; ++ci) {
                const int Y = cand[ci];
                const int X = bn / Y;
                if (X < 1 || X * Y != bn) continue;
                if (n[yi].ext % Y != 0 || n[0].ext % X != 0) continue;
                GMode x = n[0], y = n[yi];
                std::vector<GMode> rest;
                for (size_t i = 1; i < n.size(); ++i)
                    if (i != yi) rest.push_back(n[i]);
                std::vector<GMode> nn;
                nn.push_back({Y, y.i0, y.i1});
                nn.push_back({X, x.i0, x.i1});
                if (y.ext / Y > 1) nn.push_back({y.ext / Y, y.i0 * Y, y.i1 * Y});
                if (x.ext / X > 1) nn.push_back({x.ext / X, x.i0 * X, x.i1 * X});
                for (auto &r : rest) nn.push_back(r);
                n = nn;
                c.boxX = X;
                break;
            }
        }
    }
    c.m = m;
    c.n = n;
    c.k = k;
    c.M = group_size(m);
    c.N = group_size(n);
    c.K = group_size(k);
    c.h = h;
    c.H = 1;
    for (const auto &x : h) c.H *= x.ext;
    if (c.empty) c.M = c.N = c.K = c.H = 0;
    return c;
}

void output_modes(const Args &a, std::vector<int64_t> &ext, std::vector<int64_t> &inc) {
    bool skipA[kMaxRank] = {false}, skipB[kMaxRank] = {false};
    for (int64_t x = 0; x < a.conts; ++x) {
        skipA[a.conta[x]] = true;
        skipB[a.contb[x]] = true;
    }
    for (int64_t h = 0; h < a.hads; ++h) {
        skipA[a.hada[h]] = true;
        skipB[a.hadb[h]] = true;
    }
    const int64_t rc = out_rank(a);
    ext.assign(rc, 1);
    inc.assign(a.incc, a.incc + rc);
    int64_t p = 0;
    for (int64_t i = 0; i < a.ranka; ++i)
        if (!skipA[i]) ext[a.perm[p++]] = a.exta[i];
    for (int64_t j = 0; j < a.rankb; ++j)
        if (!skipB[j]) ext[a.perm[p++]] = a.extb[j];
    for (int64_t h = 0; h < a.hads; ++h) ext[a.perm[p++]] = a.exta[a.hada[h]];
}

void hadamard_offsets(const std::vector<HMode> &h, int64_t *outA, int64_t *outB, int64_t *outC) {
    int64_t total = 1;
    for (const auto &x : h) total *= x.ext;
    for (int64_t g = 0; g < total; ++g) {
        int64_t r = g, oa = 0, ob = 0, oc = 0;
        for (const auto &x : h) {
            const int64_t c = r % x.ext;
            r /= x.ext;
            oa += c * x.ia;
            ob += c * x.ib;
            oc += c * x.ic;
        }
        outA[g] = oa;
        outB[g] = ob;
        outC[g] = oc;
    }
}

void group_offsets(const std::vector<GMode> &g, int slot, int64_t padded, int64_t *out) {
    const int64_t total = group_size(g);
    std::vector<int64_t> coord(g.size(), 0);
    int64_t off = 0;
    for (int64_t idx = 0; idx < total; ++idx) {
        out[idx] = off;
        // odometer step, first mode fastest; keep the running offset
        for (size_t i = 0; i < g.size(); ++i) {
            const int64_t inc = slot ? g[i].i1 : g[i].i0;
            if (++coord[i] < g[i].ext) {
                off += inc;
                break;
            }
            off -= inc * (g[i].ext - 1);
            coord[i] = 0;
        }
    }
    for (int64_t idx = total; idx < padded; ++idx) out[idx] = 0;
}

void group_range(const std::vector<GMode> &g, int slot, int64_t &lo, int64_t &hi) {
    lo = hi = 0;
    for (const GMode &m : g) {
        const int64_t span = (slot ? m.i1 : m.i0) * (m.ext - 1);
        if (span < 0) lo += span;
        else hi += span;
    }
}

void operand_ranges(const Canon &c, int64_t &aLo, int64_t &aSpan, int64_t &bLo, int64_t &bSpan) {
    int64_t fl, fh, kl, kh;
    group_range(c.m, 0, fl, fh);
    group_range(c.k, 0, kl, kh);
    aLo = fl + kl;
    aSpan = (fh - fl) + (kh - kl);
    group_range(c.n, 0, fl, fh);
    group_range(c.k, 1, kl, kh);
    bLo = fl + kl;
    bSpan = (fh - fl) + (kh - kl);
}

void canonical_groups(const Args &a, std::vector<GMode> &rowsA, std::vector<GMode> &rowsB,
                      std::vector<GMode> &kAB) {
    raw_groups(a, rowsA, rowsB, kAB);
}

// ---------------------------------------------------------------------------
// Features for the schedule predictor (64 floats).
// ---------------------------------------------------------------------------
static float lg2(double x) { return x > 0 ? (float)std::log2(x) : 0.f; }

void features(const Args &a, int prec, float *f) {
    for (int i = 0; i < 64; ++i) f[i] = 0.f;
    Canon c = canonicalise(a, 0, 128);
    const std::vector<GMode> *groups[3] = {&c.m, &c.n, &c.k};
    int o = 0;
    for (int gi = 0; gi < 3; ++gi) {
        const auto &g = *groups[gi];
        const int64_t size = group_size(g);
        int64_t largest = 1;
        for (const auto &x : g) largest = std::max(largest, x.ext);
        const int64_t fastest = g.empty() ? 1 : g[0].ext;
        const int64_t m0 = g.empty() ? 0 : min_abs(g, 0);
        const int64_t m1 = g.empty() ? 0 : min_abs(g, 1);
        f[o + 0] = lg2((double)size);
        f[o + 1] = (float)g.size();
        f[o + 2] = lg2((double)largest);
        f[o + 3] = lg2((double)fastest);
        f[o + 4] = lg2((double)(m0 ? m0 : 1));
        f[o + 5] = lg2((double)(m1 ? m1 : 1));
        f[o + 6] = (!g.empty() && iabs(g[0].i0) == 1) ? 1.f : 0.f;
        f[o + 7] = (!g.empty() && iabs(g[0].i1) == 1) ? 1.f : 0.f;
        bool same = false;
        if (!g.empty()) {
            size_t b0 = 0, b1 = 0;
            for (size_t i = 0; i < g.size(); ++i) {
                if (iabs(g[i].i0) < iabs(g[b0].i0)) b0 = i;
                if (iabs(g[i].i1) < iabs(g[b1].i1)) b1 = i;
            }
            same = b0 == b1;
        }
        f[o + 8] = same ? 1.f : 0.f;
        f[o + 9] = (size % 16 == 0) ? 1.f : 0.f;
        f[o + 10] = (size % 64 == 0) ? 1.f : 0.f;
        f[o + 11] = (size % 128 == 0) ? 1.f : 0.f;
        o += 12;
    }
    const double M = (double)c.M, N = (double)c.N, K = (double)c.K;
    const double bytesPer = prec == 0 ? 8.0 : 4.0;
    const double flops = 2.0 * M * N * K;
    const double bytes = bytesPer * (M * K + N * K + 2.0 * M * N);
    f[o++] = lg2(flops);
    f[o++] = lg2(bytes);
    f[o++] = lg2(flops / std::max(bytes, 1.0));
    f[o++] = (float)a.ranka;
    f[o++] = (float)a.rankb;
    f[o++] = (float)(a.ranka + a.rankb - 2 * a.conts);
    f[o++] = (float)a.conts;
    for (int p = 0; p < 4; ++p) f[o++] = prec == p ? 1.f : 0.f;
    bool negA = false, negB = false, negC = false;
    for (int64_t i = 0; i < a.ranka; ++i) negA |= a.inca[i] < 0;
    for (int64_t i = 0; i < a.rankb; ++i) negB |= a.incb[i] < 0;
    for (int64_t i = 0; i < a.ranka + a.rankb - 2 * a.conts; ++i) negC |= a.incc[i] < 0;
    f[o++] = negA;
    f[o++] = negB;
    f[o++] = negC;
    f[o++] = c.swapped ? 1.f : 0.f;
    f[o++] = c.aFastK ? 1.f : 0.f;
    f[o++] = c.bFastK ? 1.f : 0.f;
    f[o++] = c.boxX ? 1.f : 0.f;
    f[o++] = lg2(std::max(M, 1.0)) - lg2(std::max(N, 1.0));
    f[o++] = lg2(std::max(M, 1.0)) - lg2(std::max(K, 1.0));
    f[o++] = lg2(std::max(N, 1.0)) - lg2(std::max(K, 1.0));
    f[o++] = (float)(std::ceil(M / 128.0) * std::ceil(N / 128.0) / 256.0);
    f[o++] = (float)(std::ceil(M / 64.0) * std::ceil(N / 64.0) / 256.0);
    // o == 62; the last two stay zero
}

std::string signature_key(const Args &a, int prec, int64_t extra0, int64_t extra1) {
    std::vector<int64_t> v;
    v.push_back(prec);
    v.push_back(extra0);
    v.push_back(extra1);
    v.push_back(a.ranka);
    for (int64_t i = 0; i < a.ranka; ++i) { v.push_back(a.exta[i]); v.push_back(a.inca[i]); }
    v.push_back(a.rankb);
    for (int64_t i = 0; i < a.rankb; ++i) { v.push_back(a.extb[i]); v.push_back(a.incb[i]); }
    v.push_back(a.conts);
    for (int64_t i = 0; i < a.conts; ++i) { v.push_back(a.conta[i]); v.push_back(a.contb[i]); }
    if (a.hads > 0) {
        v.push_back(-1 - a.hads);
        for (int64_t i = 0; i < a.hads; ++i) { v.push_back(a.hada[i]); v.push_back(a.hadb[i]); }
    }
    const int64_t rc = out_rank(a);
    for (int64_t i = 0; i < rc; ++i) { v.push_back(a.perm[i]); v.push_back(a.incc[i]); }
    return std::string(reinterpret_cast<const char *>(v.data()), v.size() * sizeof(int64_t));
}

}  // namespace gett

// Memory-safety and undefined-behaviour run of the host planner (argument
// checks, canonical M/N/K groups, offset tables, features, plan keys), built
// with AddressSanitizer and UBSan: random signatures, valid and invalid,
// with every table written into a buffer of exactly its size.  Checks the
// group sizes against the extents and that canonicalisation keeps the set of
// (A, B, C) offset triples of the contraction.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <set>
#include <tuple>
#include <vector>

#include "gett_plan.h"

using namespace gett;

static uint64_t rs = 0x9E3779B97F4A7C15ull;
static uint64_t rnd() {
    rs ^= rs << 13;
    rs ^= rs >> 7;
    rs ^= rs << 17;
    return rs;
}
static int64_t rin(int64_t lo, int64_t hi) { return lo + (int64_t)(rnd() % (uint64_t)(hi - lo + 1)); }

int main() {
    int valid = 0, invalid = 0;
    const double dummy = 0;
    for (int it = 0; it < 20000; ++it) {
        int64_t ra = rin(0, 5), rb = rin(0, 5);
        int64_t cs = rin(0, std::min(ra, rb));
        std::vector<int64_t> exta(ra), extb(rb), inca(ra), incb(rb), conta(cs), contb(cs);
        for (auto &e : exta) e = rin(1, 6);
        for (auto &e : extb) e = rin(1, 6);
        std::vector<int64_t> pa(ra), pb(rb);
        for (int64_t i = 0; i < ra; ++i) pa[i] = i;
        for (int64_t i = 0; i < rb; ++i) pb[i] = i;
        for (int64_t i = ra - 1; i > 0; --i) std::swap(pa[i], pa[rin(0, i)]);
        for (int64_t i = rb - 1; i > 0; --i) std::swap(pb[i], pb[rin(0, i)]);
        for (int64_t k = 0; k < cs; ++k) {
            conta[k] = pa[k];
            contb[k] = pb[k];
            extb[contb[k]] = exta[conta[k]];
        }
        auto strides = [](const std::vector<int64_t> &ext, std::vector<int64_t> &inc) {
            int64_t s = 1;
            for (size_t i = 0; i < ext.size(); ++i) {
                inc[i] = (rnd() & 3) ? s : -s;
                s *= ext[i] + rin(0, 1);
            }
        };
        strides(exta, inca);
        strides(extb, incb);
        const int64_t rc = ra + rb - 2 * cs;
        std::vector<int64_t> perm(rc), incc(rc);
        for (int64_t i = 0; i < rc; ++i) perm[i] = i;
        for (int64_t i = rc - 1; i > 0; --i) std::swap(perm[i], perm[rin(0, i)]);
        std::vector<int64_t> extc(rc);
        {
            int64_t p = 0;
            for (int64_t i = 0; i < ra; ++i)
                if (std::find(conta.begin(), conta.end(), i) == conta.end()) extc[perm[p++]] = exta[i];
            for (int64_t i = 0; i < rb; ++i)
                if (std::find(contb.begin(), contb.end(), i) == contb.end()) extc[perm[p++]] = extb[i];
        }
        strides(extc, incc);
        // one argument broken in a fifth of the cases
        const int broken = (rnd() % 5 == 0) ? (int)rin(1, 6) : 0;
        if (broken == 1 && ra) exta[0] = -1;
        if (broken == 2 && cs) conta[0] = ra;
        if (broken == 3 && rc > 1) perm[0] = perm[1];
        if (broken == 4 && rc && extc[0] > 1) incc[0] = 0;
        if (broken == 5 && cs) extb[contb[0]] = exta[conta[0]] + 1;
        if (broken == 6 && rb) incb[0] = INT64_MAX / 2;
        Args a{ra, exta.data(), inca.data(), rb, extb.data(), incb.data(), cs,
               conta.data(), contb.data(), perm.data(), incc.data()};
        const int info = validate(a, &dummy, &dummy, &dummy);
        if (info) {
            ++invalid;
            continue;
        }
        ++valid;
        int64_t M = 1, N = 1, K = 1;
        for (int64_t i = 0; i < ra; ++i)
            (std::find(conta.begin(), conta.end(), i) == conta.end() ? M : K) *= exta[i];
        for (int64_t i = 0; i < rb; ++i)
            if (std::find(contb.begin(), contb.end(), i) == contb.end()) N *= extb[i];
        // reference set of (offA, offB, offC) over all terms, from the arguments
        std::set<std::tuple<int64_t, int64_t, int64_t>> ref, got;
        {
            const int64_t total = M * N * K;
            if (total <= 4096) {
                std::vector<int64_t> ext;
                for (int64_t i = 0; i < ra; ++i) ext.push_back(exta[i]);
                for (int64_t i = 0; i < rb; ++i)
                    if (std::find(contb.begin(), contb.end(), i) == contb.end()) ext.push_back(extb[i]);
                std::vector<int64_t> c(ext.size(), 0);
                for (int64_t t = 0; t < total; ++t) {
                    int64_t oa = 0, ob = 0, oc = 0, p = 0, q = (int64_t)ra;
                    for (int64_t i = 0; i < ra; ++i) oa += inca[i] * c[i];
                    for (int64_t i = 0; i < rb; ++i) {
                        auto it2 = std::find(contb.begin(), contb.end(), i);
                        const int64_t ci = it2 == contb.end() ? c[q++] : c[conta[it2 - contb.begin()]];
                        ob += incb[i] * ci;
                    }
                    for (int64_t i = 0; i < ra; ++i)
                        if (std::find(conta.begin(), conta.end(), i) == conta.end()) oc += incc[perm[p++]] * c[i];
                    for (int64_t i = (int64_t)ra; i < (int64_t)c.size(); ++i) oc += incc[perm[p++]] * c[i];
                    ref.insert({oa, ob, oc});
                    for (size_t i = 0; i < c.size(); ++i) {
                        if (++c[i] < ext[i]) break;
                        c[i] = 0;
                    }
                }
            }
        }
        for (int order = 0; order < 4; ++order) {
            for (int bn : {64, 128}) {
                Canon cn = canonicalise(a, order, bn);
                if (cn.empty) continue;
                if (cn.M * cn.N * cn.K != M * N * K) return 10;
                if (!((cn.M == M && cn.N == N) || (cn.M == N && cn.N == M))) return 11;
                std::vector<int64_t> am(cn.M), cm(cn.M), bnn(cn.N), cnn(cn.N), ak(cn.K), bk(cn.K);
                group_offsets(cn.m, 0, cn.M, am.data());
                group_offsets(cn.m, 1, cn.M, cm.data());
                group_offsets(cn.n, 0, cn.N, bnn.data());
                group_offsets(cn.n, 1, cn.N, cnn.data());
                group_offsets(cn.k, 0, cn.K, ak.data());
                group_offsets(cn.k, 1, cn.K, bk.data());
                if (!ref.empty() && order == 0 && bn == 64) {
                    got.clear();
                    for (int64_t m = 0; m < cn.M; ++m)
                        for (int64_t n = 0; n < cn.N; ++n)
                            for (int64_t k = 0; k < cn.K; ++k) {
                                // swapped: the first operand is B
                                const int64_t o1 = am[m] + ak[k], o2 = bnn[n] + bk[k];
                                const int64_t oc = cm[m] + cnn[n];
                                got.insert(cn.swapped ? std::make_tuple(o2, o1, oc)
                                                      : std::make_tuple(o1, o2, oc));
                            }
                    if (got != ref) return 12;
                }
            }
        }
        std::vector<GMode> r0, r1, kk;
        canonical_groups(a, r0, r1, kk);
        int64_t s0 = 1, s1 = 1, s2 = 1;
        for (auto &x : r0) s0 *= x.ext;
        for (auto &x : r1) s1 *= x.ext;
        for (auto &x : kk) s2 *= x.ext;
        if (s0 != M || s1 != N || s2 != K) return 13;
        std::vector<int64_t> t0(s0), t1(s1), t2(s2);
        group_offsets(r0, 0, s0, t0.data());
        group_offsets(r1, 1, s1, t1.data());
        group_offsets(kk, 1, s2, t2.data());
        float f[64];
        for (int prec = 0; prec < 4; ++prec) features(a, prec, f);
        (void)signature_key(a, 2, 3, 1);
    }
    std::printf("plan fuzz: %d valid, %d rejected\n", valid, invalid);
    return valid > 5000 && invalid > 1000 ? 0 : 20;
}

// gett_host.cpp -- the C ABI of libgett.so: xGETT entry points, plan cache,
// schedule policies (heuristic, MLP predictor, autotuner) and launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "gett_bf3pack.h"
#include "gett_ozaki.h"
#include "gett.h"
#include "gett_internal.h"
#include "gett_noalloc.h"
#include "gett_plan.h"

namespace gett {

// ---------------------------------------------------------------------------
// Per-thread and global state
// ---------------------------------------------------------------------------
static thread_local hipStream_t t_stream = nullptr;
static thread_local int64_t t_last_schedule = -1;
// Initial policy from GETT_POLICY (heuristic | predict | autotune); the
// C-ABI setter overrides it.
static int policy_from_env() {
    const char *e = getenv("GETT_POLICY");
    if (!e) return GETT_HEURISTIC;
    if (strcmp(e, "predict") == 0) return GETT_PREDICT;
    if (strcmp(e, "autotune") == 0) return GETT_AUTOTUNE;
    return GETT_HEURISTIC;
}
static std::atomic<int> g_policy{policy_from_env()};
// Cap on split-K workspace bytes (GETT_MAX_WORKSPACE, gett_set_max_workspace):
// a split schedule whose FP64 partials would exceed it, or whose workspace
// cannot be allocated, runs unsplit; batches stop cutting problems along K.
static int64_t max_ws_from_env() {
    const char *e = getenv("GETT_MAX_WORKSPACE");
    if (!e || !*e) return INT64_MAX;
    char *end = nullptr;
    const long long v = strtoll(e, &end, 10);
    return (end && *end == 0 && v >= 0) ? (int64_t)v : INT64_MAX;
}
static std::atomic<int64_t> g_max_ws{max_ws_from_env()};
static std::atomic<int64_t> g_forced{-1};
static std::mutex g_mu;   // guards the caches below

static bool g_log = [] {
    const char *e = getenv("GETT_LOG");
    return e && e[0] == '1';
}();

// Device check: the kernels are built for gfx950 only.
static std::map<int, bool> g_device_ok;
static int check_device(int *dev_out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return GETT_ERR_HIP;
    *dev_out = dev;
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_device_ok.find(dev);
    if (it == g_device_ok.end()) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return GETT_ERR_HIP;
        const bool ok = strncmp(prop.gcnArchName, "gfx950", 6) == 0;
        it = g_device_ok.emplace(dev, ok).first;
    }
    return it->second ? 0 : GETT_ERR_DEVICE;
}

int current_device_checked(int *dev) { return check_device(dev); }

// ---------------------------------------------------------------------------
// Schedules
// ---------------------------------------------------------------------------
struct Sched {
    int tile, order, split;
};
static int64_t sched_id(const Sched &s) {
    return s.tile + kNumTiles * (s.order + kNumOrders * s.split);
}
static Sched sched_of(int64_t id) {
    Sched s;
    s.tile = (int)(id % kNumTiles);
    id /= kNumTiles;
    s.order = (int)(id % kNumOrders);
    s.split = (int)(id / kNumOrders);
    return s;
}
static const int64_t kNumSched = (int64_t)kNumTiles * kNumOrders * kNumSplits;

// A schedule is usable when every split gets at least one K step; the packed
// BF16x3 form takes contractions without Hadamard modes.
static bool sched_valid(int prec, const Sched &s, int64_t K, int64_t H = 1) {
    if (s.tile < 0 || s.tile >= kNumTiles || s.order < 0 || s.order >= kNumOrders || s.split < 0 ||
        s.split >= kNumSplits)
        return false;
    if (kTiles[prec][s.tile].packed && H > 1) return false;
    const int S = kSplitFactor[s.split];
    const int bk = kTiles[prec][s.tile].bk;
    if (S > 1 && K < (int64_t)S * bk) return false;
    if (S == 0 && K < 4 * (int64_t)bk) return false;     // "fill" needs a few K steps
    if (prec == kFP8 && s.split != 0) return false;
    return true;
}

// Built-in rules (the default policy, and the baseline of the predictor):
// fill the 256 CUs with whole waves of tiles, prefer larger tiles, and split
// K only when there are too few tiles to occupy the chip.
static Sched heuristic(int prec, int64_t M, int64_t N, int64_t K, int64_t H = 1) {
    // Relative per-CU throughput of each tile once the chip is full, from
    // timings of the menu on large strided and dense contractions.
    static const double kSpeed[kNumPrec][kNumTiles] = {
        {0.88, 0.92, 1.0, 0.95, 0.85},  // FP64: the 128x64 tile runs 3-4 workgroups per CU; 4 packed
        {0.8, 0.9, 0.9, 1.0, 0.95},     // FP32
        {0.7, 1.0, 0.75, 0.8, 0.9},     // BF16x3 (1 and 4: the packed form)
        {0.8, 0.9, 0.9, 1.0, 1.0},      // FP8 (its own kernel)
        {0.95, 1.0, 1.0, 0.9, 0.9},     // complex FP64
        {0.9, 0.95, 0.95, 1.0, 0.9}};   // complex FP32
    const double *kTileSpeed = kSpeed[prec];
    double best = -1;
    Sched bs{3, 0, 0};
    for (int t = 0; t < kNumTiles; ++t) {
        const TileShape ts = kTiles[prec][t];
        const double tm = std::ceil((double)M / ts.bm), tn = std::ceil((double)N / ts.bn);
        const double tiles = tm * tn * (double)std::max<int64_t>(H, 1);
        const double slots = 256.0 * ((ts.bm * ts.bn >= 128 * 128) ? 1.0 : 2.0);
        const double waves = std::ceil(tiles / slots);
        const double util = tiles / (waves * slots);
        const double pad = ((double)M / (tm * ts.bm)) * ((double)N / (tn * ts.bn));
        const double score = util * pad * kTileSpeed[t];
        if (score > best + 1e-9) {
            best = score;
            bs.tile = t;
        }
    }
    const TileShape ts = kTiles[prec][bs.tile];
    const double tiles = std::ceil((double)M / ts.bm) * std::ceil((double)N / ts.bn) *
                         (double)std::max<int64_t>(H, 1);
    bs.split = 0;
    if (prec != kFP8 && tiles < 192) {
        // too few tiles for 256 CUs: split K, as far as the contraction allows
        if (tiles <= 32 && K >= 64 * (int64_t)ts.bk) bs.split = 3;             // fill
        else if (tiles * 4 <= 512 && K >= 4 * 256) bs.split = 2;
        else if (K >= 2 * 256) bs.split = 1;
    }
    return bs;
}

// ---------------------------------------------------------------------------
// Plans
// ---------------------------------------------------------------------------
// Offset tables of one canonical form.  They depend only on the signature,
// the N-mode order and the tile width, so plans that differ in tile height,
// K step or split share them.
struct TableSet {
    Canon cn;
    int64_t Mp = 0, Np = 0, Kp = 0, Hp = 0;
    // offAM, offCM [Mp]; offBN, offCN [Np]; offAK, offBK [Kp]; then, with
    // Hadamard modes, offAH, offBH, offCH [Hp]
    int64_t *d_tab = nullptr;
    int64_t aLo = 0, aSpan = 0, bLo = 0, bSpan = 0;   // addressed element range of A and B
    int64_t cLo = 0, cSpan = 0;                        // and of C
    // Packed BF16x3 form: the rows of A, then of B, in increasing operand
    // offset (the pass whose lanes run along the rows walks them so), and
    // each one's position in the tables' order; built on first use.
    std::mutex pk_mu;
    int64_t *d_pkRows = nullptr;
    int32_t *d_pkMap = nullptr;
    ~TableSet() {
        if (d_tab) (void)hipFree(d_tab);
        if (d_pkRows) (void)hipFree(d_pkRows);
        if (d_pkMap) (void)hipFree(d_pkMap);
    }
};

struct Plan {
    int prec = 0;
    Sched sched{};
    TableSet *tab = nullptr;    // owned by g_tables
};

static std::unordered_map<std::string, std::unique_ptr<TableSet>> g_tables;
// Plans are shared: a call or a captured batch graph keeps the plans it uses
// alive while a policy change empties the cache.
static std::unordered_map<std::string, std::shared_ptr<Plan>> g_plans;

static int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Stream-ordered temporary buffers (split-K partials, packed rows, FP8
// codes, saved C footprints) come from one memory pool per device that keeps
// freed memory (release threshold: unlimited), so back-to-back calls reuse it
// instead of mapping it again; gett_finalize returns it.
static std::map<int, hipMemPool_t> g_pools;
static std::mutex g_pool_mu;

static hipMemPool_t work_pool(int dev) {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    auto it = g_pools.find(dev);
    if (it != g_pools.end()) return it->second;
    hipMemPoolProps props{};
    props.allocType = hipMemAllocationTypePinned;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = dev;
    hipMemPool_t pool = nullptr;
    if (hipMemPoolCreate(&pool, &props) != hipSuccess) {
        (void)hipGetLastError();
        pool = nullptr;
    } else {
        uint64_t keep = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    }
    g_pools[dev] = pool;
    return pool;
}

int work_alloc(void **p, size_t bytes, hipStream_t s) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return GETT_ERR_HIP;
    hipMemPool_t pool = work_pool(dev);
    const hipError_t e = pool ? hipMallocFromPoolAsync(p, bytes, pool, s) : hipMallocAsync(p, bytes, s);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return GETT_ERR_ALLOC;
    }
    return 0;
}

int work_free(void *p, hipStream_t s) { return hipFreeAsync(p, s) == hipSuccess ? 0 : GETT_ERR_HIP; }

static void work_pools_trim() {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    for (auto &kv : g_pools)
        if (kv.second) (void)hipMemPoolTrimTo(kv.second, 0);
}

// Tile width the offset tables of a schedule's tile are built for: the
// packed BF16x3 entries take the tables of their fallback tile (their GEMM
// reads packed rows, so the N order's boxes need not match its width).
static int table_bn(int prec, int tile) {
    return kTiles[prec][kTiles[prec][tile].packed ? kPackedFallbackTile : tile].bn;
}

// Build the host tables of a canonical form and upload them.
static int upload_tables(TableSet &t) {
    const Canon &c = t.cn;
    t.Mp = round_up(std::max<int64_t>(c.M, 1), kTablePad);
    t.Np = round_up(std::max<int64_t>(c.N, 1), kTablePad);
    // K tables: zero padding past K covers the kernel's look-ahead loads (two
    // steps of at most 64 positions past the last slice start, which is < K).
    t.Kp = round_up(std::max<int64_t>(c.K, 1), 128) + 256;
    t.Hp = c.H > 1 ? c.H : 0;
    std::vector<int64_t> h(2 * (t.Mp + t.Np + t.Kp) + 3 * t.Hp);
    int64_t *p = h.data();
    group_offsets(c.m, 0, t.Mp, p);
    group_offsets(c.m, 1, t.Mp, p + t.Mp);
    p += 2 * t.Mp;
    group_offsets(c.n, 0, t.Np, p);
    group_offsets(c.n, 1, t.Np, p + t.Np);
    p += 2 * t.Np;
    group_offsets(c.k, 0, t.Kp, p);
    group_offsets(c.k, 1, t.Kp, p + t.Kp);
    p += 2 * t.Kp;
    if (t.Hp) hadamard_offsets(c.h, p, p + t.Hp, p + 2 * t.Hp);
    operand_ranges(c, t.aLo, t.aSpan, t.bLo, t.bSpan);
    {
        int64_t ml, mh, nl, nh;
        group_range(c.m, 1, ml, mh);
        group_range(c.n, 1, nl, nh);
        t.cLo = ml + nl;
        t.cSpan = (mh - ml) + (nh - nl);
    }
    const size_t bytes = h.size() * sizeof(int64_t);
    if (hipMalloc(&t.d_tab, bytes) != hipSuccess) return GETT_ERR_ALLOC;
    if (hipMemcpy(t.d_tab, h.data(), bytes, hipMemcpyHostToDevice) != hipSuccess)
        return GETT_ERR_HIP;
    return 0;
}

static int get_tables(const Args &a, int order, int bn, int dev, TableSet **out) {
    const std::string key = signature_key(a, -1, dev, order * 1024 + bn);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_tables.find(key);
        if (it != g_tables.end()) {
            *out = it->second.get();
            return 0;
        }
    }
    auto t = std::make_unique<TableSet>();
    t->cn = canonicalise(a, order, bn);
    if (t->cn.M > INT32_MAX || t->cn.N > INT32_MAX || t->cn.H > INT32_MAX) return GETT_ERR_INTERNAL;
    int rc = upload_tables(*t);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_mu);
    auto &slot = g_tables[key];
    if (!slot) slot = std::move(t);
    *out = slot.get();
    return 0;
}

static Sched choose_schedule(int prec, const Args &a, int64_t M, int64_t N, int64_t K, int64_t H,
                             const char **source);

static int get_plan(int prec, const Args &a, int dev, int64_t forced, std::shared_ptr<Plan> *out) {
    const std::string key = signature_key(a, prec, dev, forced);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_plans.find(key);
        if (it != g_plans.end()) {
            *out = it->second;
            t_last_schedule = sched_id(it->second->sched);
            return 0;
        }
    }
    // Plan outside the lock (the predictor/autotuner may launch kernels).
    Canon c0 = canonicalise(a, 0, 128);
    Sched s;
    const char *source = "forced";
    if (forced >= 0) {
        s = sched_of(forced);
        if (!sched_valid(prec, s, c0.K, c0.H)) return GETT_ERR_STATE;
    } else {
        s = choose_schedule(prec, a, c0.M, c0.N, c0.K, c0.H, &source);
    }
    auto pl = std::make_shared<Plan>();
    pl->prec = prec;
    pl->sched = s;
    const TileShape ts = kTiles[prec][s.tile];
    int rc = get_tables(a, s.order, table_bn(prec, s.tile), dev, &pl->tab);
    if (rc) return rc;
    const Canon &cn = pl->tab->cn;
    const int64_t tiles = ((cn.M + ts.bm - 1) / ts.bm) * ((cn.N + ts.bn - 1) / ts.bn);
    if (tiles * split_count(s.split, tiles, std::max<int64_t>(cn.K, 1), ts.bk, nullptr) *
            std::max<int64_t>(cn.H, 1) >
        INT32_MAX)
        return GETT_ERR_INTERNAL;
    if (g_log)
        fprintf(stderr, "[gett] plan prec=%d M=%lld N=%lld K=%lld tile=%d order=%d split=%d "
                        "swapped=%d aFastK=%d bFastK=%d boxX=%d source=%s\n",
                prec, (long long)cn.M, (long long)cn.N, (long long)cn.K, s.tile, s.order, s.split,
                (int)cn.swapped, (int)cn.aFastK, (int)cn.bFastK, cn.boxX, source);
    std::lock_guard<std::mutex> lk(g_mu);
    auto &slot = g_plans[key];
    if (!slot) slot = std::move(pl);   // another thread may have won the race
    *out = slot;
    t_last_schedule = sched_id(slot->sched);
    return 0;
}

// Fill the launch parameters of a plan for concrete pointers (the plan's
// split and tile unless given).
static TileParams make_params(const Plan &pl, const void *A, const void *B, void *C,
                              int split = -1, int tile = -1) {
    const TableSet &t = *pl.tab;
    const Canon &c = t.cn;
    const TileShape ts = kTiles[pl.prec][tile < 0 ? pl.sched.tile : tile];
    if (split < 0) split = pl.sched.split;
    TileParams p;
    p.A = c.swapped ? B : A;
    p.B = c.swapped ? A : B;
    p.C = C;
    p.offAM = t.d_tab;
    p.offCM = t.d_tab + t.Mp;
    p.offBN = t.d_tab + 2 * t.Mp;
    p.offCN = t.d_tab + 2 * t.Mp + t.Np;
    p.offAK = t.d_tab + 2 * t.Mp + 2 * t.Np;
    p.offBK = t.d_tab + 2 * t.Mp + 2 * t.Np + t.Kp;
    p.M = c.M;
    p.N = c.N;
    p.K = c.K;
    p.tilesM = (int32_t)((c.M + ts.bm - 1) / ts.bm);
    p.tilesN = (int32_t)((c.N + ts.bn - 1) / ts.bn);
    int64_t per = 0;
    p.splits = split_count(split, (int64_t)p.tilesM * p.tilesN, std::max<int64_t>(c.K, 1), ts.bk,
                           &per);
    p.kPerSplit = per;
    p.bBoxX = c.boxX > 0 ? c.boxX : ts.bn;
    p.ws = nullptr;
    p.aLo = t.aLo;
    p.bLo = t.bLo;
    const int64_t esz = prec_bytes(pl.prec);
    const int64_t lim = (int64_t)1 << 32;
    p.off32 = (t.aSpan < lim / esz && t.bSpan < lim / esz) ? 1 : 0;
    p.H = (int32_t)std::max<int64_t>(c.H, 1);
    const int64_t *th = t.d_tab + 2 * (t.Mp + t.Np + t.Kp);
    // (the canonical form's Hadamard increments already follow a swap of A and B)
    p.offAH = t.Hp ? th : nullptr;
    p.offBH = t.Hp ? th + t.Hp : nullptr;
    p.offCH = t.Hp ? th + 2 * t.Hp : nullptr;
    p.alpha[0] = 1.0;
    p.alpha[1] = 0.0;
    p.beta[0] = 1.0;
    p.beta[1] = 0.0;
#ifdef GETT_ADDR_CHECK
    // GETT_CHECK_SHRINK=1 narrows the checked ranges of A and B by one
    // element at the top (the accesses themselves are unchanged), so a test
    // can see the checker report the tensors' last elements.
    static const bool shrink = [] {
        const char *e = getenv("GETT_CHECK_SHRINK");
        return e && e[0] == '1';
    }();
    p.aSpan = t.aSpan - (shrink ? 1 : 0);
    p.bSpan = t.bSpan - (shrink ? 1 : 0);
    p.cLo = t.cLo;
    p.cSpan = t.cSpan;
#endif
    return p;
}

static const double kOne[2] = {1.0, 0.0};

static int packed_rows(TableSet &t) {
    std::lock_guard<std::mutex> lk(t.pk_mu);
    if (t.d_pkRows) return 0;
    const Canon &c = t.cn;
    const int64_t R[2] = {c.M, c.N};
    std::vector<int64_t> rows(c.M + c.N);
    std::vector<int32_t> map(c.M + c.N);
    for (int side = 0; side < 2; ++side) {
        const int64_t base = side ? c.M : 0;
        std::vector<int64_t> off(R[side]);
        group_offsets(side ? c.n : c.m, 0, R[side], off.data());
        std::vector<int32_t> ord(R[side]);
        for (int64_t i = 0; i < R[side]; ++i) ord[i] = (int32_t)i;
        std::stable_sort(ord.begin(), ord.end(),
                         [&](int32_t x, int32_t y) { return off[x] < off[y]; });
        for (int64_t i = 0; i < R[side]; ++i) {
            rows[base + i] = off[ord[i]];
            map[base + i] = ord[i];
        }
    }
    const size_t n = std::max<size_t>(rows.size(), 1);
    int64_t *dr = nullptr;
    int32_t *dm = nullptr;
    if (hipMalloc(&dr, n * sizeof(int64_t)) != hipSuccess) return GETT_ERR_ALLOC;
    if (hipMalloc(&dm, n * sizeof(int32_t)) != hipSuccess) {
        (void)hipFree(dr);
        return GETT_ERR_ALLOC;
    }
    if (!rows.empty() &&
        (hipMemcpy(dr, rows.data(), rows.size() * sizeof(int64_t), hipMemcpyHostToDevice) !=
             hipSuccess ||
         hipMemcpy(dm, map.data(), map.size() * sizeof(int32_t), hipMemcpyHostToDevice) !=
             hipSuccess)) {
        (void)hipFree(dr);
        (void)hipFree(dm);
        return GETT_ERR_HIP;
    }
    t.d_pkRows = dr;
    t.d_pkMap = dm;
    return 0;
}

// The packed BF16x3 form: pack A and B into hi/lo rows (one workspace with
// the FP64 partials of a K split), the GEMM, then the slices' reduction.
// *fallback is set, with nothing launched, when the rows are too long or
// the workspace is over the cap or cannot be allocated: the caller then runs
// the direct 128 x 128 tile with the same order and split.
static int run_packed(const Plan &pl, const TileParams &p, hipStream_t s, bool *fallback) {
    *fallback = false;
    TableSet &t = *pl.tab;
    const Canon &c = t.cn;
    const bool f64 = pl.prec == kF64;
    const int64_t M = c.M, N = c.N, K = c.K;
    const TileShape ts = kTiles[pl.prec][pl.sched.tile];
    const int bk = f64 ? kPacked64BK : kPackedBK;
    const int64_t Kq = round_up(std::max<int64_t>(K, 1), bk);
    const int64_t Mq = round_up(std::max<int64_t>(M, 1), ts.bm);
    const int64_t Nq = round_up(std::max<int64_t>(N, 1), ts.bn);
    const int64_t tilesM = Mq / ts.bm, tilesN = Nq / ts.bn;
    int64_t per = 0;
    const int S = split_count(pl.sched.split, tilesM * tilesN, Kq, bk, &per);
    const int64_t pk = (f64 ? 8 : 4) * (Mq + Nq) * Kq;   // BF16x3: hi and lo bfloat16
    const int64_t wsb = S > 1 ? (int64_t)S * M * N * (int64_t)sizeof(double) : 0;
    if (Kq > kPackedMaxKq || tilesM * tilesN * S > INT32_MAX || pk + wsb > g_max_ws.load()) {
        *fallback = true;
        return 0;
    }
    int rc = packed_rows(t);
    if (rc) return rc;
    void *buf = nullptr;
    if (work_alloc(&buf, (size_t)(pk + wsb), s)) {
        *fallback = true;
        return 0;
    }
    char *PA = static_cast<char *>(buf);
    char *PB = PA + (f64 ? 8 : 4) * Mq * Kq;
    double *ws = wsb ? reinterpret_cast<double *>(static_cast<char *>(buf) + pk) : nullptr;
    rc = launch_pack(f64, p.A, c.aFastK ? p.offAM : t.d_pkRows, c.aFastK ? nullptr : t.d_pkMap, M,
                     p.offAK, K, Kq, !c.aFastK, PA, Mq * Kq, s);
    if (!rc)
        rc = launch_pack(f64, p.B, c.bFastK ? p.offBN : t.d_pkRows + M,
                         c.bFastK ? nullptr : t.d_pkMap + M, N, p.offBK, K, Kq, !c.bFastK, PB,
                         Nq * Kq, s);
    if (!rc && f64) {
        F64Packed g{};
        g.A = reinterpret_cast<const double *>(PA);
        g.B = reinterpret_cast<const double *>(PB);
        g.Kq = Kq;
        g.kPer = per;
        g.tilesM = (int32_t)tilesM;
        g.tilesN = (int32_t)tilesN;
        g.splits = S;
        g.C = static_cast<double *>(p.C);
        g.offCM = p.offCM;
        g.offCN = p.offCN;
        g.M = M;
        g.N = N;
        g.ws = ws;
        g.alpha = p.alpha[0];
        g.beta = p.beta[0];
        rc = launch_f64_packed_gemm(g, s);
    } else if (!rc) {
        Bf3Packed g{};
        g.A = reinterpret_cast<const uint16_t *>(PA);
        g.B = reinterpret_cast<const uint16_t *>(PB);
        g.planeA = Mq * Kq;
        g.planeB = Nq * Kq;
        g.Kq = Kq;
        g.kPer = per;
        g.tilesM = (int32_t)tilesM;
        g.tilesN = (int32_t)tilesN;
        g.splits = S;
        g.C = static_cast<float *>(p.C);
        g.offCM = p.offCM;
        g.offCN = p.offCN;
        g.M = M;
        g.N = N;
        g.ws = ws;
        g.alpha = p.alpha[0];
        g.beta = p.beta[0];
        rc = launch_bf3_packed_gemm(ts.bm, ts.bn, g, s);
    }
    if (!rc && S > 1) {
        TileParams q = p;
        q.ws = ws;
        q.splits = S;
        rc = launch_splitk_reduce(pl.prec, q, s);
    }
    const int frc = work_free(buf, s);
    return rc ? rc : frc;
}

// alpha, beta: (re, im) pairs of C <- alpha * sum + beta * C_in.
static int run_plan(const Plan &pl, const void *A, const void *B, void *C, hipStream_t s,
                    const double *alpha = kOne, const double *beta = kOne) {
    TileParams p = make_params(pl, A, B, C);
    auto scale = [&](TileParams &q) {
        q.alpha[0] = alpha[0];
        q.alpha[1] = alpha[1];
        q.beta[0] = beta[0];
        q.beta[1] = beta[1];
    };
    scale(p);
    int tile = pl.sched.tile;
    if (kTiles[pl.prec][tile].packed) {
        bool fallback = false;
        const int rc = run_packed(pl, p, s, &fallback);
        if (!fallback) return rc;
        tile = kPackedFallbackTile;
        t_last_schedule = sched_id(Sched{tile, pl.sched.order, pl.sched.split});
        p = make_params(pl, A, B, C, -1, tile);
        scale(p);
    }
    if (p.splits > 1) {
        const int64_t bytes = (int64_t)p.splits * p.M * p.N * (int64_t)p.H *
                              (prec_complex(pl.prec) ? 2 : 1) * (int64_t)sizeof(double);
        void *ws = nullptr;
        if (bytes <= g_max_ws.load() && work_alloc(&ws, (size_t)bytes, s) == 0) {
            p.ws = static_cast<double *>(ws);
            int rc = launch_tile(pl.prec, tile, pl.tab->cn.aFastK, pl.tab->cn.bFastK, p, s);
            if (!rc) rc = launch_splitk_reduce(pl.prec, p, s);
            const int frc = work_free(ws, s);
            return rc ? rc : frc;
        }
        // over the cap or out of memory: the same tile and order, unsplit
        (void)hipGetLastError();
        p = make_params(pl, A, B, C, 0, tile);
        scale(p);
        t_last_schedule = sched_id(Sched{tile, pl.sched.order, 0});
    }
    return launch_tile(pl.prec, tile, pl.tab->cn.aFastK, pl.tab->cn.bFastK, p, s);
}

// ---------------------------------------------------------------------------
// FP8 path
// ---------------------------------------------------------------------------
struct Fp8Plan {
    int64_t M = 0, N = 0, K = 0, nb = 0, Kp = 0;
    int64_t *d_tab = nullptr;  // rowsA [M], kA [K], rowsB [N], kB [K], offCM [M], offCN [N]
    int tile = 3;
    bool aRowsFast = false, bRowsFast = false;   // quantisation loader per operand
    bool swapped = false;      // the GEMM's first operand is B
    // For an operand quantised with lanes along its rows: its row offsets in
    // the operand's own cheapest order and, for each, the GEMM row it fills.
    int64_t *d_rowsOp[2] = {nullptr, nullptr};
    int32_t *d_rowMap[2] = {nullptr, nullptr};
    ~Fp8Plan() {
        if (d_tab) (void)hipFree(d_tab);
        for (int i = 0; i < 2; ++i) {
            if (d_rowsOp[i]) (void)hipFree(d_rowsOp[i]);
            if (d_rowMap[i]) (void)hipFree(d_rowMap[i]);
        }
    }
};
static std::unordered_map<std::string, std::unique_ptr<Fp8Plan>> g_fp8;

// Whether an operand's rows are cheaper to walk in memory than its
// contracted positions: smallest |increment| among row modes below that among
// contracted modes (slot = the operand's increment slot in the K groups).
static bool rows_fast(const std::vector<GMode> &rows, const std::vector<GMode> &k, int slot) {
    int64_t r = INT64_MAX, c = INT64_MAX;
    for (auto &x : rows)
        if (x.ext > 1) r = std::min<int64_t>(r, std::llabs(x.i0));
    for (auto &x : k)
        if (x.ext > 1) c = std::min<int64_t>(c, std::llabs(slot ? x.i1 : x.i0));
    return r < c;
}

// The rows of a group walked in the operand's own order (modes by increasing
// |operand increment|): their operand offsets, and for each the row's index
// in the group's given (GEMM) order.
static void operand_order(const std::vector<GMode> &g, int64_t R, std::vector<int64_t> &off,
                          std::vector<int32_t> &map) {
    std::vector<size_t> ord(g.size());
    for (size_t i = 0; i < g.size(); ++i) ord[i] = i;
    std::stable_sort(ord.begin(), ord.end(), [&](size_t x, size_t y) {
        return std::llabs(g[x].i0) < std::llabs(g[y].i0);
    });
    std::vector<int64_t> radix(g.size());
    int64_t r = 1;
    for (size_t i = 0; i < g.size(); ++i) {
        radix[i] = r;
        r *= g[i].ext;
    }
    std::vector<GMode> og;
    for (size_t i : ord) og.push_back(g[i]);
    off.assign(R, 0);
    group_offsets(og, 0, R, off.data());
    map.assign(R, 0);
    std::vector<int64_t> coord(og.size(), 0);
    int64_t idx = 0;   // GEMM-order index of the current operand-order row
    for (int64_t p = 0; p < R; ++p) {
        map[p] = (int32_t)idx;
        for (size_t k = 0; k < og.size(); ++k) {   // odometer, first operand-order mode fastest
            if (++coord[k] < og[k].ext) {
                idx += radix[ord[k]];
                break;
            }
            idx -= radix[ord[k]] * (og[k].ext - 1);
            coord[k] = 0;
        }
    }
}

static int get_fp8_plan(const Args &a, int dev, Fp8Plan **out) {
    const std::string key = signature_key(a, kFP8, dev, -7);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_fp8.find(key);
        if (it != g_fp8.end()) {
            *out = it->second.get();
            return 0;
        }
    }
    std::vector<GMode> ra, rb, k;
    canonical_groups(a, ra, rb, k);
    auto pl = std::make_unique<Fp8Plan>();
    // The GEMM's lanes run along N in the epilogue: when C's cheapest mode is
    // one of A's free modes, exchange the operands (the block scales are per
    // row of each operand either way, so the quantised model is unchanged).
    auto min_inc = [](const std::vector<GMode> &g, int slot) {
        int64_t m = INT64_MAX;
        for (auto &x : g)
            if (x.ext > 1) m = std::min<int64_t>(m, std::llabs(slot ? x.i1 : x.i0));
        return m;
    };
    if (min_inc(ra, 1) < min_inc(rb, 1)) {
        std::swap(ra, rb);
        for (auto &x : k) std::swap(x.i0, x.i1);
        pl->swapped = true;
    }
    // N positions in order of increasing C increment, so that the lanes of
    // the epilogue (neighbouring N positions) write neighbouring outputs.
    std::stable_sort(rb.begin(), rb.end(), [](const GMode &x, const GMode &y) {
        return std::llabs(x.i1) < std::llabs(y.i1);
    });
    auto size = [](const std::vector<GMode> &g) {
        int64_t s = 1;
        for (auto &x : g) s *= x.ext;
        return s;
    };
    pl->M = size(ra);
    pl->N = size(rb);
    pl->K = size(k);
    pl->nb = (pl->K + 127) / 128;
    pl->Kp = pl->nb * 128;
    // C offsets of the canonical rows: slot 1 of the raw M/N groups is INCC.
    std::vector<int64_t> h(2 * pl->M + 2 * pl->N + 2 * pl->K);
    int64_t *p = h.data();
    group_offsets(ra, 0, pl->M, p); p += pl->M;
    group_offsets(k, 0, pl->K, p); p += pl->K;
    group_offsets(rb, 0, pl->N, p); p += pl->N;
    group_offsets(k, 1, pl->K, p); p += pl->K;
    group_offsets(ra, 1, pl->M, p); p += pl->M;
    group_offsets(rb, 1, pl->N, p);
    const size_t bytes = h.size() * sizeof(int64_t);
    if (hipMalloc(&pl->d_tab, std::max<size_t>(bytes, 8)) != hipSuccess) return GETT_ERR_ALLOC;
    if (bytes && hipMemcpy(pl->d_tab, h.data(), bytes, hipMemcpyHostToDevice) != hipSuccess)
        return GETT_ERR_HIP;
    const int64_t tilesBig = ((pl->M + 127) / 128) * ((pl->N + 127) / 128);
    pl->tile = tilesBig >= 256 ? 3 : 0;
    pl->aRowsFast = rows_fast(ra, k, 0);
    pl->bRowsFast = rows_fast(rb, k, 1);
    for (int side = 0; side < 2; ++side) {
        const bool rf = side ? pl->bRowsFast : pl->aRowsFast;
        const std::vector<GMode> &g = side ? rb : ra;
        const int64_t R = side ? pl->N : pl->M;
        if (!rf || R == 0) continue;
        if (R > INT32_MAX) return GETT_ERR_INTERNAL;
        std::vector<int64_t> off;
        std::vector<int32_t> map;
        operand_order(g, R, off, map);
        if (hipMalloc(&pl->d_rowsOp[side], R * sizeof(int64_t)) != hipSuccess ||
            hipMalloc(&pl->d_rowMap[side], R * sizeof(int32_t)) != hipSuccess)
            return GETT_ERR_ALLOC;
        if (hipMemcpy(pl->d_rowsOp[side], off.data(), R * sizeof(int64_t),
                      hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(pl->d_rowMap[side], map.data(), R * sizeof(int32_t),
                      hipMemcpyHostToDevice) != hipSuccess)
            return GETT_ERR_HIP;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    auto &slot = g_fp8[key];
    if (!slot) slot = std::move(pl);
    *out = slot.get();
    return 0;
}

// bs: contracted positions per scale (128, or 32 for the MX-style calls);
// fmt: element format (kElemE4M3, or kElemE2M3 / kElemE2M1 with bs 32).
static int run_fp8(const Args &a, const float *A, const float *B, float *C, hipStream_t s, int dev,
                   int bs, int fmt) {
    Fp8Plan *pl = nullptr;
    int rc = get_fp8_plan(a, dev, &pl);
    if (rc) return rc;
    // The FP8 path has no schedule menu: its GEMM tile (64x64 or 128x128) is
    // chosen by tile count; reported as that tile with order and split 0.
    t_last_schedule = sched_id(Sched{pl->tile, 0, 0});
    const int64_t M = pl->M, N = pl->N, K = pl->K, nb = pl->nb, Kp = pl->Kp;
    const int64_t *rowsA = pl->d_tab, *kA = rowsA + M, *rowsB = kA + K, *kB = rowsB + N;
    const int64_t *offCM = kB + K, *offCN = offCM + M;
    const int64_t Mq = round_up(M, 128), Nq = round_up(N, 128);
    const int64_t nbs = nb * (128 / bs);   // exponents per row
    const size_t bytes = (size_t)(Mq + Nq) * Kp + (size_t)(Mq + Nq) * nbs * sizeof(int32_t) + 256;
    void *ws = nullptr;
    if (work_alloc(&ws, bytes, s)) return GETT_ERR_ALLOC;
    uint8_t *QA = static_cast<uint8_t *>(ws);
    uint8_t *QB = QA + (size_t)Mq * Kp;
    int32_t *EA = reinterpret_cast<int32_t *>(QB + (size_t)Nq * Kp);
    int32_t *EB = EA + (size_t)Mq * nbs;
    const float *X0 = pl->swapped ? B : A, *X1 = pl->swapped ? A : B;
    rc = launch_fp8_quant(X0, pl->aRowsFast ? pl->d_rowsOp[0] : rowsA, pl->d_rowMap[0], M, Mq,
                          kA, K, pl->aRowsFast, QA, EA, s, bs, fmt);
    if (!rc)
        rc = launch_fp8_quant(X1, pl->bRowsFast ? pl->d_rowsOp[1] : rowsB, pl->d_rowMap[1], N, Nq,
                              kB, K, pl->bRowsFast, QB, EB, s, bs, fmt);
    if (!rc) rc = launch_fp8_gemm(pl->tile, QA, EA, QB, EB, C, offCM, offCN, M, N, K, s, bs, fmt);
    if (work_free(ws, s) && !rc) rc = GETT_ERR_HIP;
    return rc;
}

// ---------------------------------------------------------------------------
// Predictor (MLP 64 -> 128 -> 128 -> heads tile | order | split)
// ---------------------------------------------------------------------------
struct Predictor {
    int din = 0, h1 = 0, h2 = 0, dout = 0;
    std::vector<int64_t> heads;
    std::vector<float> mean, stdv;
    float *d_w = nullptr;   // W1 b1 W2 b2 W3 b3 contiguous
    float *d_io = nullptr;  // x [din], y1 [h1], y2 [h2], z [dout]
    size_t off[6] = {0, 0, 0, 0, 0, 0};
    int dev = -1;
    ~Predictor() {
        if (d_w) (void)hipFree(d_w);
        if (d_io) (void)hipFree(d_io);
    }
};
static std::unique_ptr<Predictor> g_pred;
static std::mutex g_pred_mu;

static int load_predictor(const char *path) {
    FILE *f = fopen(path, "rb");
    if (!f) return GETT_ERR_STATE;
    char magic[8];
    int32_t dims[5];
    auto pred = std::make_unique<Predictor>();
    bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, "GETTMLP1", 8) == 0 &&
              fread(dims, 4, 5, f) == 5;
    if (ok) {
        pred->din = dims[0];
        pred->h1 = dims[1];
        pred->h2 = dims[2];
        pred->dout = dims[3];
        const int nh = dims[4];
        ok = pred->din == GETT_NUM_FEATURES && nh == 3 && pred->h1 > 0 && pred->h2 > 0 &&
             pred->h1 <= 4096 && pred->h2 <= 4096;
        std::vector<int32_t> hs(3);
        ok = ok && fread(hs.data(), 4, 3, f) == 3;
        if (ok) {
            pred->heads.assign(hs.begin(), hs.end());
            ok = hs[0] == kNumTiles && hs[1] == kNumOrders && hs[2] == kNumSplits &&
                 hs[0] + hs[1] + hs[2] == pred->dout;
        }
    }
    std::vector<float> w;
    if (ok) {
        pred->mean.resize(pred->din);
        pred->stdv.resize(pred->din);
        ok = fread(pred->mean.data(), 4, pred->din, f) == (size_t)pred->din &&
             fread(pred->stdv.data(), 4, pred->din, f) == (size_t)pred->din;
        const size_t sizes[6] = {(size_t)pred->h1 * pred->din, (size_t)pred->h1,
                                 (size_t)pred->h2 * pred->h1, (size_t)pred->h2,
                                 (size_t)pred->dout * pred->h2, (size_t)pred->dout};
        size_t total = 0;
        for (int i = 0; i < 6; ++i) {
            pred->off[i] = total;
            total += sizes[i];
        }
        w.resize(total);
        ok = ok && fread(w.data(), 4, total, f) == total;
    }
    fclose(f);
    if (!ok) return GETT_ERR_STATE;
    if (hipGetDevice(&pred->dev) != hipSuccess) return GETT_ERR_HIP;
    if (hipMalloc(&pred->d_w, w.size() * 4) != hipSuccess) return GETT_ERR_ALLOC;
    if (hipMemcpy(pred->d_w, w.data(), w.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
        return GETT_ERR_HIP;
    if (hipMalloc(&pred->d_io, (size_t)(pred->din + pred->h1 + pred->h2 + pred->dout) * 4) !=
        hipSuccess)
        return GETT_ERR_ALLOC;
    std::lock_guard<std::mutex> lk(g_pred_mu);
    g_pred = std::move(pred);
    return 0;
}

// Run the network on one feature vector with the library's own kernels and
// return the best valid joint schedule under the summed log-probabilities.
// A schedule filter (nullptr: every valid schedule of the menu).
typedef bool (*SchedFilter)(int prec, const Sched &s);

static bool predict(int prec, const Args &a, int64_t K, Sched *out, SchedFilter allow = nullptr) {
    // Without a loaded network, GETT_MODEL names the weights file to load
    // (once, on the first prediction).
    static std::once_flag env_model;
    std::call_once(env_model, [] {
        const char *m = getenv("GETT_MODEL");
        bool have;
        {
            std::lock_guard<std::mutex> lk(g_pred_mu);
            have = g_pred != nullptr;
        }
        if (m && !have && load_predictor(m) != 0 && g_log)
            fprintf(stderr, "[gett] GETT_MODEL=%s could not be loaded\n", m);
    });
    std::lock_guard<std::mutex> lk(g_pred_mu);
    Predictor *pr = g_pred.get();
    if (!pr) return false;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev != pr->dev) return false;
    float feat[GETT_NUM_FEATURES];
    features(a, prec, feat);
    for (int i = 0; i < pr->din; ++i)
        feat[i] = (feat[i] - pr->mean[i]) / (pr->stdv[i] > 0 ? pr->stdv[i] : 1.f);
    float *x = pr->d_io, *y1 = x + pr->din, *y2 = y1 + pr->h1, *z = y2 + pr->h2;
    hipStream_t s = t_stream;
    if (hipMemcpyAsync(x, feat, pr->din * 4, hipMemcpyHostToDevice, s) != hipSuccess) return false;
    const float *W = pr->d_w;
    if (launch_mlp_linear_fwd(x, W + pr->off[0], W + pr->off[1], y1, 1, pr->din, pr->h1, 1, s) ||
        launch_mlp_linear_fwd(y1, W + pr->off[2], W + pr->off[3], y2, 1, pr->h1, pr->h2, 1, s) ||
        launch_mlp_linear_fwd(y2, W + pr->off[4], W + pr->off[5], z, 1, pr->h2, pr->dout, 0, s))
        return false;
    std::vector<float> logits(pr->dout);
    if (hipMemcpyAsync(logits.data(), z, pr->dout * 4, hipMemcpyDeviceToHost, s) != hipSuccess)
        return false;
    if (hipStreamSynchronize(s) != hipSuccess) return false;
    // log-softmax per head
    std::vector<double> lp(pr->dout);
    int o = 0;
    for (int h = 0; h < 3; ++h) {
        const int n = (int)pr->heads[h];
        double mx = -1e300;
        for (int i = 0; i < n; ++i) mx = std::max(mx, (double)logits[o + i]);
        double se = 0;
        for (int i = 0; i < n; ++i) se += std::exp((double)logits[o + i] - mx);
        for (int i = 0; i < n; ++i) lp[o + i] = (double)logits[o + i] - mx - std::log(se);
        o += n;
    }
    double best = -1e300;
    bool found = false;
    for (int64_t id = 0; id < kNumSched; ++id) {
        Sched sc = sched_of(id);
        if (!sched_valid(prec, sc, K) || (allow && !allow(prec, sc))) continue;
        const double v = lp[sc.tile] + lp[kNumTiles + sc.order] + lp[kNumTiles + kNumOrders + sc.split];
        if (v > best) {
            best = v;
            *out = sc;
            found = true;
        }
    }
    return found;
}

// ---------------------------------------------------------------------------
// Autotuner
// ---------------------------------------------------------------------------
static int time_schedule(int prec, const Args &a, const void *A, const void *B, void *C, int dev,
                         int64_t id, int warmup, int reps, double *us) {
    std::shared_ptr<Plan> pl;
    int rc = get_plan(prec, a, dev, id, &pl);
    if (rc) return rc;
    hipStream_t s = t_stream;
    for (int i = 0; i < warmup; ++i)
        if ((rc = run_plan(*pl, A, B, C, s))) return rc;
    std::vector<double> t(reps);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return GETT_ERR_HIP;
    for (int r = 0; r < reps; ++r) {
        (void)hipEventRecord(e0, s);
        rc = run_plan(*pl, A, B, C, s);
        (void)hipEventRecord(e1, s);
        if (rc) break;
        if (hipEventSynchronize(e1) != hipSuccess) { rc = GETT_ERR_HIP; break; }
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        t[r] = ms * 1e3;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    std::sort(t.begin(), t.end());
    *us = t[reps / 2];
    return 0;
}

// HBM bytes a schedule is modelled to move: each tile reads its A rows and
// B columns over its K range (a panel is fetched again by every tile row or
// column that needs it), C is read and written once, and a K split writes
// and reads back its FP64 partials.
static double modeled_bytes(int prec, const Canon &c, Sched s) {
    const TileShape ts = kTiles[prec][s.tile];
    const int64_t tm = (c.M + ts.bm - 1) / ts.bm, tn = (c.N + ts.bn - 1) / ts.bn;
    const int S = split_count(s.split, tm * tn, std::max<int64_t>(c.K, 1), ts.bk, nullptr);
    const double esz = (double)prec_bytes(prec), mn = (double)c.M * (double)c.N * (double)c.H;
    double b = (double)tm * (double)tn * (double)(ts.bm + ts.bn) * (double)c.K * (double)c.H * esz +
               2.0 * mn * esz;
    if (S > 1) b += 2.0 * S * mn * (prec_complex(prec) ? 16.0 : 8.0);
    return b;
}

// Two passes: every valid schedule once (after `warmup` untimed runs), then
// the fastest few again, `reps` timed runs each after one untimed run; their
// medians decide.  The second pass runs in rounds that time every candidate
// once, so a drift of the clock or power state over the pass shifts all
// candidates alike instead of favouring the ones timed first.  times[]
// receives the median for re-timed schedules, the single time for the
// others, and -1 for invalid ones.  With prefer_less_traffic the pick among
// the re-timed schedules within kTieWindow of the fastest median is the one
// with the fewest modelled HBM bytes (the medians of the best few often lie
// within the timing noise of one another; the one that moves less data keeps
// more of its speed under sustained load); otherwise the fastest median.
constexpr double kTieWindow = 0.02;
static int64_t autotune(int prec, const Args &a, const void *A, const void *B, void *C, int dev,
                        int warmup, int reps, double *times, int64_t ntimes, int *status,
                        SchedFilter allow = nullptr, bool prefer_less_traffic = false) {
    Canon c0 = canonicalise(a, 0, 128);
    *status = 0;
    std::vector<double> t1(kNumSched, -1.0);
    for (int64_t id = 0; id < kNumSched; ++id) {
        if (!sched_valid(prec, sched_of(id), c0.K, c0.H) || (allow && !allow(prec, sched_of(id))))
            continue;
        int rc = time_schedule(prec, a, A, B, C, dev, id, warmup, 1, &t1[id]);
        if (rc) {
            *status = rc;
            return -1;
        }
    }
    std::vector<int64_t> order;
    for (int64_t id = 0; id < kNumSched; ++id)
        if (t1[id] > 0) order.push_back(id);
    std::sort(order.begin(), order.end(), [&](int64_t x, int64_t y) { return t1[x] < t1[y]; });
    const size_t top = std::min<size_t>(order.size(), 6);
    if (top == 0) return -1;
    std::vector<std::shared_ptr<Plan>> plans(top);
    hipStream_t s = t_stream;
    int rc = 0;
    for (size_t i = 0; i < top && !rc; ++i)
        if (!(rc = get_plan(prec, a, dev, order[i], &plans[i]))) rc = run_plan(*plans[i], A, B, C, s);
    if (rc) {
        *status = rc;
        return -1;
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) {
        *status = GETT_ERR_HIP;
        return -1;
    }
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        *status = GETT_ERR_HIP;
        return -1;
    }
    const int nr = std::max(reps, 1);
    std::vector<std::vector<double>> tt(top, std::vector<double>(nr));
    for (int r = 0; r < nr && !rc; ++r)
        for (size_t i = 0; i < top && !rc; ++i) {
            (void)hipEventRecord(e0, s);
            rc = run_plan(*plans[i], A, B, C, s);
            (void)hipEventRecord(e1, s);
            if (rc) break;
            if (hipEventSynchronize(e1) != hipSuccess) {
                rc = GETT_ERR_HIP;
                break;
            }
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            tt[i][r] = ms * 1e3;
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) {
        *status = rc;
        return -1;
    }
    double best = 1e300;
    int64_t best_id = -1;
    for (size_t i = 0; i < top; ++i) {
        std::sort(tt[i].begin(), tt[i].end());
        const double us = tt[i][nr / 2];
        t1[order[i]] = us;
        if (us < best) {
            best = us;
            best_id = order[i];
        }
    }
    if (prefer_less_traffic) {
        double least = modeled_bytes(prec, c0, sched_of(best_id));
        for (size_t i = 0; i < top; ++i) {
            const int64_t id = order[i];
            if (t1[id] > best * (1.0 + kTieWindow)) continue;
            const double b = modeled_bytes(prec, c0, sched_of(id));
            if (b < least) {
                least = b;
                best_id = id;
            }
        }
    }
    if (times)
        for (int64_t id = 0; id < kNumSched && id < ntimes; ++id) times[id] = t1[id];
    return best_id;
}

// Tuned choices found by the AUTOTUNE policy (signature -> schedule).
static std::unordered_map<std::string, Sched> g_tuned;

// The same choices persisted across processes when GETT_TUNE_DB names a
// file: one text line per signature, its integers (precision, then the
// xGETT arguments), " = ", the schedule id and its median time in
// microseconds.  The file is read on the first tuning decision and a line is
// appended after each new tuning; a later line for the same signature wins,
// and lines that do not parse or name an invalid schedule are ignored.
static std::unordered_map<std::string, Sched> g_tuned_db;
static bool g_tuned_db_read = false;

static const char *tune_db_path() {
    const char *p = getenv("GETT_TUNE_DB");
    return (p && *p) ? p : nullptr;
}

static std::string tune_db_key(const Args &a, int prec) {
    const std::string bin = signature_key(a, prec, -1, -3);
    std::string s;
    for (size_t i = 0; i < bin.size() / sizeof(int64_t); ++i) {
        int64_t v;
        memcpy(&v, bin.data() + i * sizeof(int64_t), sizeof v);
        if (i) s += ' ';
        s += std::to_string(v);
    }
    return s;
}

static void read_tune_db_locked() {
    if (g_tuned_db_read) return;
    g_tuned_db_read = true;
    const char *path = tune_db_path();
    FILE *f = path ? fopen(path, "r") : nullptr;
    if (!f) return;   // no file yet
    char *line = nullptr;
    size_t cap = 0;
    while (getline(&line, &cap, f) > 0) {
        const char *eq = strstr(line, " = ");
        long long id = -1;
        if (!eq || sscanf(eq + 3, "%lld", &id) != 1 || id < 0 || id >= kNumSched) continue;
        g_tuned_db[std::string(line, eq - line)] = sched_of(id);
    }
    free(line);
    fclose(f);
}

static void append_tune_db_locked(const std::string &key, int64_t id, double us) {
    const char *path = tune_db_path();
    FILE *f = path ? fopen(path, "a") : nullptr;
    if (!f) return;
    fprintf(f, "%s = %lld %.3f\n", key.c_str(), (long long)id, us);
    fclose(f);
}

static thread_local const void *t_tune_ptrs[3] = {nullptr, nullptr, nullptr};
static thread_local int t_tune_dev = 0;

static Sched choose_schedule(int prec, const Args &a, int64_t M, int64_t N, int64_t K, int64_t H,
                             const char **source) {
    const int pol = g_policy.load();
    Sched s = heuristic(prec, M, N, K, H);
    *source = "heuristic";
    // The predictor knows the real precisions of single contractions only.
    if (pol == GETT_PREDICT && prec <= kFP8 && a.hads == 0) {
        Sched p;
        if (predict(prec, a, K, &p)) {
            s = p;
            *source = "predictor";
        }
    } else if (pol == GETT_AUTOTUNE && t_tune_ptrs[0]) {
        const std::string key = signature_key(a, prec, t_tune_dev, -3);
        const std::string dkey = tune_db_key(a, prec);
        {
            std::lock_guard<std::mutex> lk(g_mu);
            auto it = g_tuned.find(key);
            if (it != g_tuned.end()) {
                *source = "tuned";
                return it->second;
            }
            read_tune_db_locked();
            auto jt = g_tuned_db.find(dkey);
            if (jt != g_tuned_db.end() && sched_valid(prec, jt->second, K, H)) {
                g_tuned[key] = jt->second;
                *source = "tune-db";
                return jt->second;
            }
        }
        int st = 0;
        // The tuning runs accumulate into C; run() saves and restores C's
        // footprint around a plan-cache miss under this policy.
        std::vector<double> us(kNumSched, -1.0);
        const int64_t id = autotune(prec, a, t_tune_ptrs[0], t_tune_ptrs[1],
                                    const_cast<void *>(t_tune_ptrs[2]), t_tune_dev, 1, 5,
                                    us.data(), kNumSched, &st, nullptr, true);
        if (!st && id >= 0) {
            s = sched_of(id);
            *source = "autotuned";
            std::lock_guard<std::mutex> lk(g_mu);
            g_tuned[key] = s;
            g_tuned_db[dkey] = s;
            append_tune_db_locked(dkey, id, us[id]);
        }
    }
    return s;
}

// ---------------------------------------------------------------------------
// Entry point shared by the single-problem calls
// ---------------------------------------------------------------------------
static int64_t c_span_elems(const Args &a, int64_t *lo_out) {
    // extent of C's footprint in elements: [lo, hi]
    std::vector<int64_t> extc, incc;
    output_modes(a, extc, incc);
    int64_t lo = 0, hi = 0;
    for (size_t q = 0; q < extc.size(); ++q) {
        if (extc[q] <= 1) continue;
        const int64_t d = incc[q] * (extc[q] - 1);
        if (d < 0) lo += d;
        else hi += d;
    }
    *lo_out = lo;
    return hi - lo + 1;
}

// C <- beta * C_in on every output (the scaled calls whose contracted sum is
// empty: a contracted extent of zero).
static int scale_outputs(int prec, const Args &a, void *C, const double *beta, hipStream_t s) {
    std::vector<int64_t> extc, incc;
    output_modes(a, extc, incc);
    ScaleModes sm{};
    sm.total = 1;
    for (size_t q = 0; q < extc.size(); ++q) {
        sm.total *= extc[q];
        if (extc[q] == 1) continue;
        if (sm.n >= kScaleModes) return GETT_ERR_INTERNAL;
        sm.ext[sm.n] = extc[q];
        sm.inc[sm.n] = incc[q];
        ++sm.n;
    }
    if (sm.total == 0) return 0;
    return launch_scale_c(prec, C, sm, beta, s);
}

static bool is_one(const double *x) { return x[0] == 1.0 && x[1] == 0.0; }

// alpha, beta: (re, im) pairs of C <- alpha * sum + beta * C_in (kOne for
// the paper's accumulate).
static int run(int prec, const Args &a, const void *A, const void *B, void *C,
               const double *alpha = kOne, const double *beta = kOne, int fp8_block = 128,
               int fp8_fmt = kElemE4M3) {
    int info = validate(a, A, B, C);
    if (info) return info;
    Canon probe = canonicalise(a, 0, 128);
    if (probe.empty || probe.M == 0 || probe.N == 0 || probe.K == 0 || probe.H == 0) {
        // No term at all.  The paper's accumulate leaves C as it is; a scaled
        // call still scales C_in (by beta) wherever C has outputs.
        if (is_one(beta)) return 0;
        int dev = 0;
        int rc = check_device(&dev);
        if (rc) return rc;
        return scale_outputs(prec, a, C, beta, t_stream);
    }
    int dev = 0;
    int rc = check_device(&dev);
    if (rc) return rc;
    hipStream_t s = t_stream;
    if (prec == kFP8)
        return run_fp8(a, static_cast<const float *>(A), static_cast<const float *>(B),
                       static_cast<float *>(C), s, dev, fp8_block, fp8_fmt);
    const int64_t forced = g_forced.load();
    std::shared_ptr<Plan> pl;
    // Under the AUTOTUNE policy a plan-cache miss times the menu; the timing
    // runs accumulate into C, so C's footprint is saved and restored around it
    // (only then: a cached plan needs no timing).
    void *saved = nullptr;
    int64_t lo = 0, span = 0;
    const size_t esz = (size_t)prec_bytes(prec);
    bool cached = false;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        cached = g_plans.count(signature_key(a, prec, dev, forced)) != 0;
    }
    if (g_policy.load() == GETT_AUTOTUNE && forced < 0 && !cached) {
        span = c_span_elems(a, &lo);
        char *cbase = static_cast<char *>(C) + lo * (int64_t)esz;
        if (hipMallocAsync(&saved, span * esz, s) != hipSuccess) return GETT_ERR_ALLOC;
        if (hipMemcpyAsync(saved, cbase, span * esz, hipMemcpyDeviceToDevice, s) != hipSuccess)
            return GETT_ERR_HIP;
        t_tune_ptrs[0] = A;
        t_tune_ptrs[1] = B;
        t_tune_ptrs[2] = C;
        t_tune_dev = dev;
    }
    rc = get_plan(prec, a, dev, forced, &pl);
    t_tune_ptrs[0] = nullptr;
    if (saved) {
        char *cbase = static_cast<char *>(C) + lo * (int64_t)esz;
        if (hipMemcpyAsync(cbase, saved, span * esz, hipMemcpyDeviceToDevice, s) != hipSuccess &&
            !rc)
            rc = GETT_ERR_HIP;
        (void)hipFreeAsync(saved, s);
    }
    if (rc) return rc;
    return run_plan(*pl, A, B, C, s, alpha, beta);
}

// ---------------------------------------------------------------------------
// DGETT emulated on INT8 matrix cores (Ozaki scheme, gett_ozaki.hip)
// ---------------------------------------------------------------------------
static int run_ozaki(const Args &a, const double *A, const double *B, double *C, int slices) {
    int info = validate(a, A, B, C);
    if (info) return info;
    if (slices < kOzMinSlices || slices > kOzMaxSlices) return GETT_ERR_STATE;
    Canon probe = canonicalise(a, 0, 128);
    if (probe.empty || probe.M == 0 || probe.N == 0 || probe.K == 0) return 0;
    int dev = 0;
    int rc = check_device(&dev);
    if (rc) return rc;
    hipStream_t s = t_stream;
    Fp8Plan *pl = nullptr;   // the canonical rows and their walk orders
    rc = get_fp8_plan(a, dev, &pl);
    if (rc) return rc;
    t_last_schedule = -1;
    const int64_t M = pl->M, N = pl->N, K = pl->K;
    const int64_t *rowsA = pl->d_tab, *kA = rowsA + M, *rowsB = kA + K, *kB = rowsB + N;
    const int64_t *offCM = kB + K, *offCN = offCM + M;
    const int64_t Kq = round_up(K, 64), Mq = round_up(M, 64), Nq = round_up(N, 64);
    // K slices of at most kOzMaxKSlice positions (the INT32 sums stay exact)
    int64_t nks = (Kq + kOzMaxKSlice - 1) / kOzMaxKSlice;
    const int64_t per = round_up((Kq + nks - 1) / nks, 64);
    nks = (Kq + per - 1) / per;
    const int64_t tilesM = Mq / 64, tilesN = Nq / 64;
    if (tilesM * tilesN * nks > INT32_MAX) return GETT_ERR_INTERNAL;
    const int64_t planeA = Mq * Kq, planeB = Nq * Kq;
    const int64_t qbytes = round_up((int64_t)slices * (planeA + planeB), 256);
    const int64_t ebytes = round_up((Mq + Nq) * (int64_t)sizeof(int32_t), 256);
    const int64_t wsb = nks > 1 ? nks * M * N * (int64_t)sizeof(double) : 0;
    void *ws = nullptr;
    if (work_alloc(&ws, (size_t)(qbytes + ebytes + wsb), s)) return GETT_ERR_ALLOC;
    uint8_t *QA = static_cast<uint8_t *>(ws);
    uint8_t *QB = QA + slices * planeA;
    int32_t *EA = reinterpret_cast<int32_t *>(static_cast<char *>(ws) + qbytes);
    int32_t *EB = EA + Mq;
    double *part = wsb ? reinterpret_cast<double *>(static_cast<char *>(ws) + qbytes + ebytes)
                       : nullptr;
    OzOperand oa{pl->swapped ? B : A, pl->aRowsFast ? pl->d_rowsOp[0] : rowsA, pl->d_rowMap[0],
                 M, kA, K, pl->aRowsFast};
    OzOperand ob{pl->swapped ? A : B, pl->bRowsFast ? pl->d_rowsOp[1] : rowsB, pl->d_rowMap[1],
                 N, kB, K, pl->bRowsFast};
    rc = launch_oz_exponents(oa, Kq, EA, Mq, s);
    if (!rc) rc = launch_oz_exponents(ob, Kq, EB, Nq, s);
    if (!rc) rc = launch_oz_slices(slices, oa, Kq, QA, planeA, EA, s);
    if (!rc) rc = launch_oz_slices(slices, ob, Kq, QB, planeB, EB, s);
    if (!rc) {
        OzParams g{};
        g.A = QA;
        g.B = QB;
        g.planeA = planeA;
        g.planeB = planeB;
        g.EA = EA;
        g.EB = EB;
        g.Kq = Kq;
        g.kPer = per;
        g.tilesM = (int32_t)tilesM;
        g.tilesN = (int32_t)tilesN;
        g.splits = (int32_t)nks;
        g.C = C;
        g.offCM = offCM;
        g.offCN = offCN;
        g.M = M;
        g.N = N;
        g.ws = part;
        rc = launch_oz_gemm(slices, g, s);
    }
    if (!rc && nks > 1) {
        // C <- C_in + sum of the K slices' FP64 values, in slice order
        TileParams q{};
        q.C = C;
        q.offCM = offCM;
        q.offCN = offCN;
        q.M = M;
        q.N = N;
        q.splits = (int32_t)nks;
        q.H = 1;
        q.ws = part;
        q.alpha[0] = q.beta[0] = 1.0;
        rc = launch_splitk_reduce(kF64, q, s);
    }
    if (work_free(ws, s) && !rc) rc = GETT_ERR_HIP;
    return rc;
}

// ---------------------------------------------------------------------------
// Allocation-free DGETT: tables and split-K partials in the device scratch
// array (gett_noalloc.hip); no plan cache, no allocation of any kind on the
// device.
// ---------------------------------------------------------------------------
static void fill_group(const std::vector<GMode> &g, int idx, int64_t size, int64_t pad,
                       FillGroups &f) {
    f.nmodes[idx] = (int32_t)g.size();
    for (size_t j = 0; j < g.size(); ++j) f.modes[idx][j] = FillMode{g[j].ext, g[j].i0, g[j].i1};
    f.size[idx] = size;
    f.pad[idx] = pad;
}

static int run_noalloc(const Args &a, const double *A, const double *B, double *C) {
    int info = validate(a, A, B, C);
    if (info) return info;
    Canon probe = canonicalise(a, 0, 128);
    if (probe.empty || probe.M == 0 || probe.N == 0 || probe.K == 0) return 0;
    const int64_t forced = g_forced.load();
    Sched s = forced >= 0 ? sched_of(forced) : heuristic(kF64, probe.M, probe.N, probe.K);
    if (!sched_valid(kF64, s, probe.K)) return GETT_ERR_STATE;
    // the packed form needs a workspace for its rows: its fallback tile runs
    if (kTiles[kF64][s.tile].packed) s.tile = kPackedFallbackTile;
    const TileShape ts = kTiles[kF64][s.tile];
    // The plan, built on the stack: canonical form, padded table lengths and
    // address ranges as in a cached plan, tables in the scratch array.
    TableSet t;
    t.cn = canonicalise(a, s.order, ts.bn);
    const Canon &c = t.cn;
    if (c.M > INT32_MAX || c.N > INT32_MAX) return GETT_ERR_INTERNAL;
    if ((int)c.m.size() > kFillModes || (int)c.n.size() > kFillModes ||
        (int)c.k.size() > kFillModes)
        return GETT_ERR_SCRATCH;
    t.Mp = round_up(std::max<int64_t>(c.M, 1), kTablePad);
    t.Np = round_up(std::max<int64_t>(c.N, 1), kTablePad);
    t.Kp = round_up(std::max<int64_t>(c.K, 1), 128) + 256;
    const int64_t tab_bytes = round_up(2 * (t.Mp + t.Np + t.Kp) * (int64_t)sizeof(int64_t), 256);
    if (tab_bytes > (int64_t)GETT_NOALLOC_SCRATCH_BYTES) return GETT_ERR_SCRATCH;
    operand_ranges(c, t.aLo, t.aSpan, t.bLo, t.bSpan);
    {
        int64_t ml, mh, nl, nh;
        group_range(c.m, 1, ml, mh);
        group_range(c.n, 1, nl, nh);
        t.cLo = ml + nl;
        t.cSpan = (mh - ml) + (nh - nl);
    }
    const int64_t tiles = ((c.M + ts.bm - 1) / ts.bm) * ((c.N + ts.bn - 1) / ts.bn);
    if (tiles * split_count(s.split, tiles, std::max<int64_t>(c.K, 1), ts.bk, nullptr) >
        INT32_MAX)
        return GETT_ERR_INTERNAL;
    int dev = 0;
    int rc = check_device(&dev);
    if (rc) return rc;
    void *scr = nullptr;
    int64_t scr_bytes = 0;
    rc = noalloc_scratch(dev, &scr, &scr_bytes);
    if (rc) return rc;
    hipStream_t st = t_stream;
    FillGroups f{};
    fill_group(c.m, 0, c.M, t.Mp, f);
    fill_group(c.n, 1, c.N, t.Np, f);
    fill_group(c.k, 2, c.K, t.Kp, f);
    int64_t *tab = static_cast<int64_t *>(scr);
    rc = launch_table_fill(f, tab, st);
    if (rc) return rc;
    t.d_tab = tab;
    Plan pl;
    pl.prec = kF64;
    pl.sched = s;
    pl.tab = &t;
    TileParams p = make_params(pl, A, B, C);
    t_last_schedule = sched_id(s);
    if (p.splits > 1) {
        const int64_t ws_bytes = (int64_t)p.splits * p.M * p.N * (int64_t)sizeof(double);
        if (tab_bytes + ws_bytes <= scr_bytes) {
            // every (slice, m, n) partial is written by its tile: no clearing
            p.ws = reinterpret_cast<double *>(static_cast<char *>(scr) + tab_bytes);
            rc = launch_tile(kF64, s.tile, c.aFastK, c.bFastK, p, st);
            if (!rc) rc = launch_splitk_reduce(kF64, p, st);
        } else {
            p = make_params(pl, A, B, C, 0);
            t_last_schedule = sched_id(Sched{s.tile, s.order, 0});
            rc = launch_tile(kF64, s.tile, c.aFastK, c.bFastK, p, st);
        }
    } else {
        rc = launch_tile(kF64, s.tile, c.aFastK, c.bFastK, p, st);
    }
    t.d_tab = nullptr;   // the scratch array is not the table set's to free
    return rc;
}

// ---------------------------------------------------------------------------
// Batches
// ---------------------------------------------------------------------------
struct BatchGraph {
    // Two instances of the graph, each copying its own pinned descriptor
    // buffer: the host fills one while the GPU may still be running the
    // replay that copied the other.
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    BatchProblem *h_desc[2] = {nullptr, nullptr};   // pinned host descriptors
    hipEvent_t done[2] = {nullptr, nullptr};         // replay of instance b finished
    int next = 0;                                    // instance of the next replay
    BatchProblem *d_desc = nullptr;
    int32_t *d_items = nullptr;
    int32_t nprobs = 0, nitems = 0;
    std::vector<std::shared_ptr<Plan>> plans;
    std::vector<int64_t> sids;   // each problem's schedule (-1: nothing to compute)
    // Problems cut along K: slice count, slice length and workspace offset
    // (doubles) per problem (splits 1: not cut), the list of cut problems on
    // the device and their FP64 partial-sum workspace.
    std::vector<int32_t> splits;
    std::vector<int64_t> kper, ws_off;
    int32_t *d_split = nullptr;
    double *d_ws = nullptr;
    std::mutex mu;             // one caller at a time rewrites and launches
    ~BatchGraph() {
        for (int b = 0; b < 2; ++b) {
            if (exec[b]) (void)hipGraphExecDestroy(exec[b]);
            if (graph[b]) (void)hipGraphDestroy(graph[b]);
            if (h_desc[b]) (void)hipHostFree(h_desc[b]);
            if (done[b]) (void)hipEventDestroy(done[b]);
        }
        if (d_desc) (void)hipFree(d_desc);
        if (d_items) (void)hipFree(d_items);
        if (d_split) (void)hipFree(d_split);
        if (d_ws) (void)hipFree(d_ws);
    }
};
static std::unordered_map<std::string, std::unique_ptr<BatchGraph>> g_graphs;

// Schedules of the problems of the calling thread's last batch (-1: empty).
static thread_local std::vector<int64_t> t_batch_scheds;

static int batch_tile_index(int prec, int tile) {
    for (int b = 0; b < kBatchTiles; ++b)
        if (kBatchTile[prec][b] == tile) return b;
    return -1;
}

// Schedules a batch problem can run: a batch tile, any N order, K unsplit
// (the batch cuts long contractions itself).
static bool batch_allow(int prec, const Sched &s) {
    return s.split == 0 && batch_tile_index(prec, s.tile) >= 0;
}

// Built-in choice for a batch problem: the batch tile whose tiles waste the
// least padding, weighted by the tile's relative speed (the batch as a whole
// fills the chip, so the tile need not), N order by C's strides (the
// epilogue's stores coalesce: on the uneven 512-problem batch the order by
// C measured 3 % faster than the order by B, and the tile choice within
// 1 %, the replay being bound by the latency of its many short items).
static Sched batch_heuristic(int prec, int64_t M, int64_t N) {
    static const double kBatchSpeed[kNumPrec][kBatchTiles] = {
        {0.9, 1.0}, {0.9, 1.0}, {0.95, 1.0}, {1, 1}, {1, 1}, {1, 1}};
    Sched best{kBatchTile[prec][0], 1, 0};
    double bs = -1;
    for (int b = 0; b < kBatchTiles; ++b) {
        const TileShape ts = kTiles[prec][kBatchTile[prec][b]];
        const double pad = ((double)M / (std::ceil((double)M / ts.bm) * ts.bm)) *
                           ((double)N / (std::ceil((double)N / ts.bn) * ts.bn));
        const double score = pad * kBatchSpeed[prec][b];
        if (score > bs + 1e-9) {
            bs = score;
            best.tile = kBatchTile[prec][b];
        }
    }
    return best;
}

// The schedule one problem of a batch runs, under the current policy: a
// forced schedule that a batch can run; else the heuristic, the predictor or
// the autotuner restricted to the batch's schedules (the autotuner times the
// problem alone, with C's footprint saved and restored around the timing).
static int batch_schedule(int prec, const Args &a, const void *A, const void *B, void *C,
                          int dev, hipStream_t st, int64_t *id_out) {
    const Canon c0 = canonicalise(a, 0, 128);
    const int64_t forced = g_forced.load();
    if (forced >= 0 && batch_allow(prec, sched_of(forced)) &&
        sched_valid(prec, sched_of(forced), c0.K)) {
        *id_out = forced;
        return 0;
    }
    Sched s = batch_heuristic(prec, c0.M, c0.N);
    const int pol = g_policy.load();
    if (pol == GETT_PREDICT && prec <= kFP8) {
        Sched ps;
        if (predict(prec, a, c0.K, &ps, batch_allow)) s = ps;
    } else if (pol == GETT_AUTOTUNE) {
        int64_t lo = 0;
        const int64_t span = c_span_elems(a, &lo);
        const size_t esz = (size_t)prec_bytes(prec);
        char *cbase = static_cast<char *>(C) + lo * (int64_t)esz;
        void *saved = nullptr;
        if (hipMallocAsync(&saved, span * esz, st) != hipSuccess) return GETT_ERR_ALLOC;
        int rc = hipMemcpyAsync(saved, cbase, span * esz, hipMemcpyDeviceToDevice, st) !=
                         hipSuccess
                     ? GETT_ERR_HIP
                     : 0;
        int status = 0;
        int64_t id = -1;
        if (!rc) id = autotune(prec, a, A, B, C, dev, 1, 5, nullptr, 0, &status, batch_allow);
        if (hipMemcpyAsync(cbase, saved, span * esz, hipMemcpyDeviceToDevice, st) !=
                hipSuccess &&
            !rc)
            rc = GETT_ERR_HIP;
        (void)hipFreeAsync(saved, st);
        if (rc) return rc;
        if (status) return status;
        if (id >= 0) s = sched_of(id);
    }
    *id_out = sched_id(s);
    return 0;
}

// Run a batch: per-problem plans with the batch tile (64x64 of the precision),
// problems with long contractions cut along K, one work list ordered longest
// item first, and a graph of {descriptor copy, persistent kernel, reduction
// of the cut problems} captured once per batch signature and replayed.  Pointers may change between calls: the descriptors are rewritten
// in pinned memory (after the previous replay has finished) before each
// replay, and the graph's copy node moves them to the device.
static int run_batch(int prec, int64_t count, const Args *args, const void *const *A,
                     const void *const *B, void *const *C, int dev, hipStream_t s) {
    std::string key;
    key.reserve(64 * count);
    key.append(reinterpret_cast<const char *>(&prec), sizeof prec);
    key.append(reinterpret_cast<const char *>(&dev), sizeof dev);
    // the per-problem schedules depend on the policy and a forced schedule
    const int64_t pol_key[2] = {(int64_t)g_policy.load(), g_forced.load()};
    key.append(reinterpret_cast<const char *>(pol_key), sizeof pol_key);
    std::vector<char> live(count, 0);
    for (int64_t i = 0; i < count; ++i) {
        // a problem with a zero extent anywhere has nothing to compute
        bool nz = true;
        for (int64_t j = 0; j < args[i].ranka; ++j) nz = nz && args[i].exta[j] != 0;
        for (int64_t j = 0; j < args[i].rankb; ++j) nz = nz && args[i].extb[j] != 0;
        live[i] = nz;
        key += signature_key(args[i], prec, live[i], 0);
    }
    BatchGraph *bg = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_graphs.find(key);
        if (it != g_graphs.end()) bg = it->second.get();
    }
    if (!bg) {
        auto nb = std::make_unique<BatchGraph>();
        nb->plans.assign(count, nullptr);
        nb->splits.assign(count, 1);
        nb->kper.assign(count, 0);
        nb->ws_off.assign(count, 0);
        nb->sids.assign(count, -1);
        const int grid_max = std::max(batch_grid_size(prec), 1);
        // Work of an item in steps of the 64 x 64 tile: a step of a larger
        // tile counts its area over 64 x 64.
        auto area = [&](const Plan &pl) {
            const TileShape ts = kTiles[prec][pl.sched.tile];
            return (double)(ts.bm * ts.bn) / (64.0 * 64.0);
        };
        // Work in K steps per problem; a problem whose tiles would each take
        // more steps than the average workgroup's share (at least 64) is cut
        // along K into slices of about that length, so no single item holds
        // up the whole launch.  Slices write FP64 partials that a reduction
        // kernel in the same graph adds to C_in in slice order.
        double total = 0;
        for (int64_t i = 0; i < count; ++i) {
            if (!live[i]) continue;
            int rc = batch_schedule(prec, args[i], A[i], B[i], C[i], dev, s, &nb->sids[i]);
            if (rc) return rc;
            std::shared_ptr<Plan> pl;
            rc = get_plan(prec, args[i], dev, nb->sids[i], &pl);
            if (rc) return rc;
            nb->plans[i] = pl;
            TileParams p = make_params(*pl, nullptr, nullptr, nullptr);
            const int bk = kTiles[prec][pl->sched.tile].bk;
            total += (double)p.tilesM * p.tilesN * ((p.K + bk - 1) / bk) * area(*pl);
        }
        const double cap = std::max(64.0, total / grid_max);
        struct Work { int64_t len; int32_t prob, nitems; };
        std::vector<Work> work;
        std::vector<int32_t> cut;
        int64_t ws_total = 0;
        for (int64_t i = 0; i < count; ++i) {
            if (!nb->plans[i]) continue;
            TileParams p = make_params(*nb->plans[i], nullptr, nullptr, nullptr);
            const int bk = kTiles[prec][nb->plans[i]->sched.tile].bk;
            const double ar = area(*nb->plans[i]);
            const int64_t steps = (p.K + bk - 1) / bk;
            int64_t S = 1, per = steps * bk;
            if (steps * ar > cap) {
                S = (int64_t)std::ceil(steps * ar / cap);
                per = (steps + S - 1) / S * bk;
                S = (p.K + per - 1) / per;      // every slice starts below K
                if ((ws_total + S * p.M * p.N) * (int64_t)sizeof(double) > g_max_ws.load()) {
                    S = 1;                       // over the workspace cap: not cut
                    per = steps * bk;
                }
            }
            const int64_t items = (int64_t)p.tilesM * p.tilesN * S;
            if (items > INT32_MAX / 2) return GETT_ERR_INTERNAL;
            if (S > 1) {
                nb->splits[i] = (int32_t)S;
                nb->kper[i] = per;
                nb->ws_off[i] = ws_total;
                ws_total += S * p.M * p.N;
                cut.push_back((int32_t)i);
            }
            work.push_back({(int64_t)((S > 1 ? per : p.K) * ar), (int32_t)i, (int32_t)items});
        }
        std::stable_sort(work.begin(), work.end(),
                         [](const Work &a, const Work &b) { return a.len > b.len; });
        std::vector<int32_t> items;
        for (auto &w : work)
            for (int32_t t = 0; t < w.nitems; ++t) {
                items.push_back(w.prob);
                items.push_back(t);
            }
        if (ws_total > 0 &&
            (hipMalloc(reinterpret_cast<void **>(&nb->d_ws), ws_total * sizeof(double)) !=
                 hipSuccess ||
             hipMalloc(reinterpret_cast<void **>(&nb->d_split), cut.size() * sizeof(int32_t)) !=
                 hipSuccess))
            return GETT_ERR_ALLOC;
        if (!cut.empty() && hipMemcpy(nb->d_split, cut.data(), cut.size() * sizeof(int32_t),
                                      hipMemcpyHostToDevice) != hipSuccess)
            return GETT_ERR_HIP;
        nb->nprobs = (int32_t)count;
        nb->nitems = (int32_t)(items.size() / 2);
        // The descriptors, then the batch kernel's item counter: each replay's
        // copy of the pinned buffer (whose counter word stays 0) clears it.
        const size_t desc_bytes = sizeof(BatchProblem) * std::max<int64_t>(count, 1);
        const size_t dbytes = desc_bytes + 256;
        if (hipMalloc(reinterpret_cast<void **>(&nb->d_desc), dbytes) != hipSuccess ||
            hipMalloc(reinterpret_cast<void **>(&nb->d_items),
                      std::max<size_t>(items.size(), 2) * sizeof(int32_t)) != hipSuccess)
            return GETT_ERR_ALLOC;
        if (!items.empty() &&
            hipMemcpy(nb->d_items, items.data(), items.size() * sizeof(int32_t),
                      hipMemcpyHostToDevice) != hipSuccess)
            return GETT_ERR_HIP;
        const int grid = std::min<int64_t>(grid_max, std::max<int32_t>(nb->nitems, 1));
        for (int b = 0; b < 2; ++b) {
            if (hipHostMalloc(reinterpret_cast<void **>(&nb->h_desc[b]), dbytes,
                              hipHostMallocDefault) != hipSuccess)
                return GETT_ERR_ALLOC;
            memset(nb->h_desc[b], 0, dbytes);
            if (hipEventCreateWithFlags(&nb->done[b], hipEventDisableTiming) != hipSuccess)
                return GETT_ERR_HIP;
            hipStream_t cs;
            if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)
                return GETT_ERR_HIP;
            int rc = 0;
            if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess)
                rc = GETT_ERR_HIP;
            if (!rc && hipMemcpyAsync(nb->d_desc, nb->h_desc[b], dbytes, hipMemcpyHostToDevice,
                                      cs) != hipSuccess)
                rc = GETT_ERR_HIP;
            if (!rc && nb->nitems > 0)
                rc = launch_batch(prec, nb->d_desc, nb->nprobs, nb->d_items, nb->nitems,
                                  reinterpret_cast<int32_t *>(
                                      reinterpret_cast<char *>(nb->d_desc) + desc_bytes),
                                  grid, cs);
            if (!rc && !cut.empty())
                rc = launch_batch_reduce(prec, nb->d_desc, nb->d_split, (int32_t)cut.size(), cs);
            hipGraph_t g = nullptr;
            if (hipStreamEndCapture(cs, &g) != hipSuccess && !rc) rc = GETT_ERR_HIP;
            nb->graph[b] = g;
            if (!rc && hipGraphInstantiate(&nb->exec[b], g, nullptr, nullptr, 0) != hipSuccess)
                rc = GETT_ERR_HIP;
            (void)hipStreamDestroy(cs);
            if (rc) return rc;
        }
        std::lock_guard<std::mutex> lk(g_mu);
        auto &slot = g_graphs[key];
        if (!slot) slot = std::move(nb);
        bg = slot.get();
    }
    // The replay that last used this instance's pinned descriptors (two
    // replays ago) must have finished before they are rewritten.
    std::lock_guard<std::mutex> lk(bg->mu);
    const int b = bg->next;
    bg->next ^= 1;
    if (hipEventSynchronize(bg->done[b]) != hipSuccess) return GETT_ERR_HIP;
    BatchProblem *h = bg->h_desc[b];
    for (int64_t i = 0; i < count; ++i) {
        if (!bg->plans[i]) continue;
        const Plan &pl = *bg->plans[i];
        h[i].p = make_params(pl, A[i], B[i], C[i]);
        if (bg->splits[i] > 1) {
            h[i].p.splits = bg->splits[i];
            h[i].p.kPerSplit = bg->kper[i];
            h[i].p.ws = bg->d_ws + bg->ws_off[i];
        }
        h[i].aFastK = pl.tab->cn.aFastK;
        h[i].bFastK = pl.tab->cn.bFastK;
        h[i].tsel = batch_tile_index(prec, pl.sched.tile);
    }
    t_batch_scheds = bg->sids;
    // Replays share the device descriptors and workspace: order this one
    // after the previous replay even when the caller switched streams.
    if (hipStreamWaitEvent(s, bg->done[b ^ 1], 0) != hipSuccess) return GETT_ERR_HIP;
    if (hipGraphLaunch(bg->exec[b], s) != hipSuccess) return GETT_ERR_HIP;
    if (hipEventRecord(bg->done[b], s) != hipSuccess) return GETT_ERR_HIP;
    return 0;
}

static int batch_entry(int prec, int64_t count, const int64_t *ranka, const int64_t *const *exta,
                       const int64_t *const *inca, const void *const *A, const int64_t *rankb,
                       const int64_t *const *extb, const int64_t *const *incb,
                       const void *const *B, const int64_t *conts,
                       const int64_t *const *conta, const int64_t *const *contb,
                       const int64_t *const *perm, const int64_t *const *incc, void *const *C,
                       int64_t *info) {
    if (count < 0) return -1;
    if (prec != kF64 && prec != kF32 && prec != kBF3) return -2;
    if (count == 0) return 0;
    if (!ranka || !exta || !inca || !A || !rankb || !extb || !incb || !B || !conts || !conta ||
        !contb || !perm || !incc || !C)
        return -1;
    std::vector<Args> args(count);
    int first_bad = 0;
    for (int64_t i = 0; i < count; ++i) {
        args[i] = Args{ranka[i], exta[i], inca[i], rankb[i], extb[i], incb[i], conts[i],
                       conta[i], contb[i], perm[i], incc[i]};
        const int v = validate(args[i], A[i], B[i], C[i]);
        if (info) info[i] = v;
        if (v && !first_bad) first_bad = (int)(-1000 * (i + 1) + v);
    }
    if (first_bad) return first_bad;
    int dev = 0;
    int rc = check_device(&dev);
    if (rc) return rc;
    return run_batch(prec, count, args.data(), A, B, C, dev, t_stream);
}

}  // namespace gett

namespace gett {
// INFO of the scaled calls, numbered in their argument order
// (ALPHA, RANKA, EXTA, INCA, A, RANKB, EXTB, INCB, B, CONTS, CONTA, CONTB,
// HADS, HADA, HADB, PERM, INCC, BETA, C): codes of the 14-argument checks
// move to their new positions.
static int ex_info(int v) {
    if (v == 0) return 0;
    if (v == kInfoHads) return -13;
    if (v == kInfoHada) return -14;
    if (v == kInfoHadb) return -15;
    if (v >= -11) return v - 1;       // RANKA .. CONTB
    if (v == -12) return -16;         // PERM
    if (v == -13) return -17;         // INCC
    return -19;                       // C
}

static int run_ex(int prec, const double *alpha, const Args &a, const void *A, const void *B,
                  void *C, const double *beta) {
    const int info = ex_info(validate(a, A, B, C));
    if (info) return info;
    return run(prec, a, A, B, C, alpha, beta);
}
}  // namespace gett

using namespace gett;

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
#define GETT_ARGS_DECL                                                                          \
    int64_t ranka, const int64_t *exta, const int64_t *inca, int64_t rankb,                     \
        const int64_t *extb, const int64_t *incb, int64_t conts, const int64_t *conta,          \
        const int64_t *contb, const int64_t *perm, const int64_t *incc
#define GETT_ARGS_MAKE Args{ranka, exta, inca, rankb, extb, incb, conts, conta, contb, perm, incc}

extern "C" {

int dgett(int64_t ranka, const int64_t *exta, const int64_t *inca, const double *A, int64_t rankb,
          const int64_t *extb, const int64_t *incb, const double *B, int64_t conts,
          const int64_t *conta, const int64_t *contb, const int64_t *perm, const int64_t *incc,
          double *C) {
    return run(kF64, GETT_ARGS_MAKE, A, B, C);
}

int sgett(int64_t ranka, const int64_t *exta, const int64_t *inca, const float *A, int64_t rankb,
          const int64_t *extb, const int64_t *incb, const float *B, int64_t conts,
          const int64_t *conta, const int64_t *contb, const int64_t *perm, const int64_t *incc,
          float *C) {
    return run(kF32, GETT_ARGS_MAKE, A, B, C);
}

int sgett_bf16x3(int64_t ranka, const int64_t *exta, const int64_t *inca, const float *A,
                 int64_t rankb, const int64_t *extb, const int64_t *incb, const float *B,
                 int64_t conts, const int64_t *conta, const int64_t *contb, const int64_t *perm,
                 const int64_t *incc, float *C) {
    return run(kBF3, GETT_ARGS_MAKE, A, B, C);
}

int sgett_fp8(int64_t ranka, const int64_t *exta, const int64_t *inca, const float *A,
              int64_t rankb, const int64_t *extb, const int64_t *incb, const float *B,
              int64_t conts, const int64_t *conta, const int64_t *contb, const int64_t *perm,
              const int64_t *incc, float *C) {
    return run(kFP8, GETT_ARGS_MAKE, A, B, C);
}

int dgett_ozaki(int64_t ranka, const int64_t *exta, const int64_t *inca, const double *A,
                int64_t rankb, const int64_t *extb, const int64_t *incb, const double *B,
                int64_t conts, const int64_t *conta, const int64_t *contb, const int64_t *perm,
                const int64_t *incc, double *C, int64_t slices) {
    return run_ozaki(GETT_ARGS_MAKE, A, B, C, (int)std::min<int64_t>(std::max<int64_t>(slices, 0), 64));
}

static int fp8_quantize_entry(int64_t rankx, const int64_t *extx, const int64_t *incx,
                              const float *X, int64_t conts, const int64_t *contx, uint8_t *QX,
                              int32_t *EX, int bs, int fmt) {
    if (rankx < 0 || rankx > 64) return -1;
    if (rankx > 0 && !extx) return -2;
    int64_t n = 1;
    for (int64_t i = 0; i < rankx; ++i) {
        if (extx[i] < 0) return -2;
        n *= extx[i];
    }
    if (rankx > 0 && !incx) return -3;
    if (n > 0 && !X) return -4;
    if (conts < 0 || conts > rankx) return -5;
    if (conts > 0 && !contx) return -6;
    bool used[64] = {false};
    for (int64_t k = 0; k < conts; ++k) {
        if (contx[k] < 0 || contx[k] >= rankx || used[contx[k]]) return -6;
        used[contx[k]] = true;
    }
    std::vector<GMode> rows, kk;
    for (int64_t i = 0; i < rankx; ++i)
        if (!used[i]) rows.push_back({extx[i], incx[i], 0});
    for (int64_t k = 0; k < conts; ++k) kk.push_back({extx[contx[k]], incx[contx[k]], 0});
    int64_t R = 1, K = 1;
    for (auto &x : rows) R *= x.ext;
    for (auto &x : kk) K *= x.ext;
    if (R * K > 0 && (!QX)) return -7;
    if (R * K > 0 && (!EX)) return -8;
    if (R == 0 || K == 0) return 0;
    int dev = 0;
    int rc = check_device(&dev);
    if (rc) return rc;
    std::vector<int64_t> h(R + K);
    group_offsets(rows, 0, R, h.data());
    group_offsets(kk, 0, K, h.data() + R);
    int64_t *d = nullptr;
    hipStream_t s = t_stream;
    if (hipMallocAsync(reinterpret_cast<void **>(&d), h.size() * 8, s) != hipSuccess)
        return GETT_ERR_ALLOC;
    if (hipMemcpyAsync(d, h.data(), h.size() * 8, hipMemcpyHostToDevice, s) != hipSuccess)
        return GETT_ERR_HIP;
    rc = launch_fp8_quant(X, d, nullptr, R, R, d + R, K, rows_fast(rows, kk, 0), QX, EX, s, bs,
                          fmt);
    (void)hipFreeAsync(d, s);
    // h must outlive the copy: wait for it
    if (hipStreamSynchronize(s) != hipSuccess && !rc) rc = GETT_ERR_HIP;
    return rc;
}

int sgett_fp8_quantize(int64_t rankx, const int64_t *extx, const int64_t *incx, const float *X,
                       int64_t conts, const int64_t *contx, uint8_t *QX, int32_t *EX) {
    return fp8_quantize_entry(rankx, extx, incx, X, conts, contx, QX, EX, 128, kElemE4M3);
}

int sgett_mxfp8_quantize(int64_t rankx, const int64_t *extx, const int64_t *incx, const float *X,
                         int64_t conts, const int64_t *contx, uint8_t *QX, int32_t *EX) {
    return fp8_quantize_entry(rankx, extx, incx, X, conts, contx, QX, EX, 32, kElemE4M3);
}

int sgett_mxfp6_quantize(int64_t rankx, const int64_t *extx, const int64_t *incx, const float *X,
                         int64_t conts, const int64_t *contx, uint8_t *QX, int32_t *EX) {
    return fp8_quantize_entry(rankx, extx, incx, X, conts, contx, QX, EX, 32, kElemE2M3);
}

int sgett_mxfp4_quantize(int64_t rankx, const int64_t *extx, const int64_t *incx, const float *X,
                         int64_t conts, const int64_t *contx, uint8_t *QX, int32_t *EX) {
    return fp8_quantize_entry(rankx, extx, incx, X, conts, contx, QX, EX, 32, kElemE2M1);
}

int sgett_mxfp8(int64_t ranka, const int64_t *exta, const int64_t *inca, const float *A,
                int64_t rankb, const int64_t *extb, const int64_t *incb, const float *B,
                int64_t conts, const int64_t *conta, const int64_t *contb, const int64_t *perm,
                const int64_t *incc, float *C) {
    return run(kFP8, GETT_ARGS_MAKE, A, B, C, kOne, kOne, 32, kElemE4M3);
}

int sgett_mxfp6(int64_t ranka, const int64_t *exta, const int64_t *inca, const float *A,
                int64_t rankb, const int64_t *extb, const int64_t *incb, const float *B,
                int64_t conts, const int64_t *conta, const int64_t *contb, const int64_t *perm,
                const int64_t *incc, float *C) {
    return run(kFP8, GETT_ARGS_MAKE, A, B, C, kOne, kOne, 32, kElemE2M3);
}

int sgett_mxfp4(int64_t ranka, const int64_t *exta, const int64_t *inca, const float *A,
                int64_t rankb, const int64_t *extb, const int64_t *incb, const float *B,
                int64_t conts, const int64_t *conta, const int64_t *contb, const int64_t *perm,
                const int64_t *incc, float *C) {
    return run(kFP8, GETT_ARGS_MAKE, A, B, C, kOne, kOne, 32, kElemE2M1);
}

int sgett_batch(int64_t count, int64_t prec, const int64_t *ranka, const int64_t *const *exta,
                const int64_t *const *inca, const float *const *A, const int64_t *rankb,
                const int64_t *const *extb, const int64_t *const *incb, const float *const *B,
                const int64_t *conts, const int64_t *const *conta, const int64_t *const *contb,
                const int64_t *const *perm, const int64_t *const *incc, float *const *C,
                int64_t *info) {
    if (prec != GETT_FP32 && prec != GETT_BF16X3) return count < 0 ? -1 : -2;
    return batch_entry((int)prec, count, ranka, exta, inca, reinterpret_cast<const void *const *>(A),
                       rankb, extb, incb, reinterpret_cast<const void *const *>(B), conts, conta,
                       contb, perm, incc, reinterpret_cast<void *const *>(C), info);
}

int dgett_batch(int64_t count, int64_t prec, const int64_t *ranka, const int64_t *const *exta,
                const int64_t *const *inca, const double *const *A, const int64_t *rankb,
                const int64_t *const *extb, const int64_t *const *incb, const double *const *B,
                const int64_t *conts, const int64_t *const *conta, const int64_t *const *contb,
                const int64_t *const *perm, const int64_t *const *incc, double *const *C,
                int64_t *info) {
    (void)prec;
    return batch_entry(kF64, count, ranka, exta, inca, reinterpret_cast<const void *const *>(A),
                       rankb, extb, incb, reinterpret_cast<const void *const *>(B), conts, conta,
                       contb, perm, incc, reinterpret_cast<void *const *>(C), info);
}

int zgett(int64_t ranka, const int64_t *exta, const int64_t *inca, const void *A, int64_t rankb,
          const int64_t *extb, const int64_t *incb, const void *B, int64_t conts,
          const int64_t *conta, const int64_t *contb, const int64_t *perm, const int64_t *incc,
          void *C) {
    return run(kZ64, GETT_ARGS_MAKE, A, B, C);
}

int cgett(int64_t ranka, const int64_t *exta, const int64_t *inca, const void *A, int64_t rankb,
          const int64_t *extb, const int64_t *incb, const void *B, int64_t conts,
          const int64_t *conta, const int64_t *contb, const int64_t *perm, const int64_t *incc,
          void *C) {
    return run(kC32, GETT_ARGS_MAKE, A, B, C);
}

int dgett_noalloc(int64_t ranka, const int64_t *exta, const int64_t *inca, const double *A,
                  int64_t rankb, const int64_t *extb, const int64_t *incb, const double *B,
                  int64_t conts, const int64_t *conta, const int64_t *contb, const int64_t *perm,
                  const int64_t *incc, double *C) {
    return run_noalloc(GETT_ARGS_MAKE, A, B, C);
}

#define GETT_EX_ARGS_MAKE                                                                        \
    Args{ranka, exta, inca, rankb, extb, incb, conts, conta, contb, perm, incc, hads, hada, hadb}

int dgett_ex(double alpha, int64_t ranka, const int64_t *exta, const int64_t *inca,
             const double *A, int64_t rankb, const int64_t *extb, const int64_t *incb,
             const double *B, int64_t conts, const int64_t *conta, const int64_t *contb,
             int64_t hads, const int64_t *hada, const int64_t *hadb, const int64_t *perm,
             const int64_t *incc, double beta, double *C) {
    const double al[2] = {alpha, 0.0}, be[2] = {beta, 0.0};
    return run_ex(kF64, al, GETT_EX_ARGS_MAKE, A, B, C, be);
}

int sgett_ex(float alpha, int64_t ranka, const int64_t *exta, const int64_t *inca,
             const float *A, int64_t rankb, const int64_t *extb, const int64_t *incb,
             const float *B, int64_t conts, const int64_t *conta, const int64_t *contb,
             int64_t hads, const int64_t *hada, const int64_t *hadb, const int64_t *perm,
             const int64_t *incc, float beta, float *C) {
    const double al[2] = {alpha, 0.0}, be[2] = {beta, 0.0};
    return run_ex(kF32, al, GETT_EX_ARGS_MAKE, A, B, C, be);
}

int sgett_bf16x3_ex(float alpha, int64_t ranka, const int64_t *exta, const int64_t *inca,
                    const float *A, int64_t rankb, const int64_t *extb, const int64_t *incb,
                    const float *B, int64_t conts, const int64_t *conta, const int64_t *contb,
                    int64_t hads, const int64_t *hada, const int64_t *hadb,
                    const int64_t *perm, const int64_t *incc, float beta, float *C) {
    const double al[2] = {alpha, 0.0}, be[2] = {beta, 0.0};
    return run_ex(kBF3, al, GETT_EX_ARGS_MAKE, A, B, C, be);
}

int zgett_ex(const double *alpha, int64_t ranka, const int64_t *exta, const int64_t *inca,
             const void *A, int64_t rankb, const int64_t *extb, const int64_t *incb,
             const void *B, int64_t conts, const int64_t *conta, const int64_t *contb,
             int64_t hads, const int64_t *hada, const int64_t *hadb, const int64_t *perm,
             const int64_t *incc, const double *beta, void *C) {
    if (!alpha) return -1;
    if (!beta) return -18;
    return run_ex(kZ64, alpha, GETT_EX_ARGS_MAKE, A, B, C, beta);
}

int cgett_ex(const float *alpha, int64_t ranka, const int64_t *exta, const int64_t *inca,
             const void *A, int64_t rankb, const int64_t *extb, const int64_t *incb,
             const void *B, int64_t conts, const int64_t *conta, const int64_t *contb,
             int64_t hads, const int64_t *hada, const int64_t *hadb, const int64_t *perm,
             const int64_t *incc, const float *beta, void *C) {
    if (!alpha) return -1;
    if (!beta) return -18;
    const double al[2] = {alpha[0], alpha[1]}, be[2] = {beta[0], beta[1]};
    return run_ex(kC32, al, GETT_EX_ARGS_MAKE, A, B, C, be);
}

int gett_set_stream(void *hip_stream) {
    t_stream = static_cast<hipStream_t>(hip_stream);
    return 0;
}
void *gett_get_stream(void) { return t_stream; }

int gett_set_policy(int policy) {
    if (policy < GETT_HEURISTIC || policy > GETT_AUTOTUNE) return GETT_ERR_STATE;
    g_policy.store(policy);
    std::lock_guard<std::mutex> lk(g_mu);
    g_plans.clear();     // plans were chosen under the old policy
    return 0;
}
int gett_get_policy(void) { return g_policy.load(); }

int gett_load_predictor(const char *path) { return path ? load_predictor(path) : GETT_ERR_STATE; }

int64_t gett_num_tiles(int prec) { return (prec >= 0 && prec < kNumPrec) ? kNumTiles : 0; }

int gett_tile_shape(int prec, int64_t t, int64_t *out) {
    if (prec < 0 || prec >= kNumPrec || t < 0 || t >= kNumTiles || !out) return GETT_ERR_STATE;
    out[0] = kTiles[prec][t].bm;
    out[1] = kTiles[prec][t].bn;
    out[2] = kTiles[prec][t].bk;
    return 0;
}

int gett_set_schedule(int64_t id) {
    if (id >= kNumSched) return GETT_ERR_STATE;
    g_forced.store(id < 0 ? -1 : id);
    return 0;
}
int64_t gett_last_schedule(void) { return t_last_schedule; }

int64_t gett_batch_last_schedules(int64_t *ids, int64_t n) {
    const int64_t m = (int64_t)t_batch_scheds.size();
    if (ids)
        for (int64_t i = 0; i < n && i < m; ++i) ids[i] = t_batch_scheds[i];
    return m;
}

int64_t gett_addr_violations(int reset) {
#ifdef GETT_ADDR_CHECK
    int64_t total = 0;
    for (int prec : {kF64, kF32, kBF3, kZ64, kC32}) {
        const int64_t v = addr_violations(prec, reset != 0);
        if (v < 0) return GETT_ERR_HIP;
        total += v;
    }
    return total;
#else
    (void)reset;
    return -1;
#endif
}

int gett_set_max_workspace(int64_t bytes) {
    if (bytes < 0) return GETT_ERR_STATE;
    g_max_ws.store(bytes);
    return 0;
}

int64_t gett_autotune(int prec, int64_t ranka, const int64_t *exta, const int64_t *inca,
                      const void *A, int64_t rankb, const int64_t *extb, const int64_t *incb,
                      const void *B, int64_t conts, const int64_t *conta, const int64_t *contb,
                      const int64_t *perm, const int64_t *incc, void *C, int64_t warmup,
                      int64_t reps, double *times_us, int64_t ntimes, int *status) {
    int st = 0;
    if (!status) status = &st;
    if (prec < 0 || prec > 2 || reps < 1 || warmup < 0) {
        *status = GETT_ERR_STATE;
        return -1;
    }
    Args a = GETT_ARGS_MAKE;
    int info = validate(a, A, B, C);
    if (info) {
        *status = info;
        return -1;
    }
    Canon c = canonicalise(a, 0, 128);
    if (c.empty || c.M * c.N * c.K == 0) {
        *status = GETT_ERR_STATE;
        return -1;
    }
    int dev = 0;
    int rc = check_device(&dev);
    if (rc) {
        *status = rc;
        return -1;
    }
    return autotune(prec, a, A, B, C, dev, (int)warmup, (int)reps, times_us, ntimes, status);
}

int64_t gett_heuristic_schedule(int prec, GETT_ARGS_DECL) {
    Args a = GETT_ARGS_MAKE;
    const int info = validate(a, reinterpret_cast<void *>(1), reinterpret_cast<void *>(1),
                              reinterpret_cast<void *>(1));
    if (info) return info;
    if (prec < 0 || prec > 3) return GETT_ERR_STATE;
    Canon c = canonicalise(a, 0, 128);
    return sched_id(heuristic(prec, c.M, c.N, c.K));
}

int gett_features(int prec, GETT_ARGS_DECL, float *out) {
    Args a = GETT_ARGS_MAKE;
    const int info = validate(a, reinterpret_cast<void *>(1), reinterpret_cast<void *>(1),
                              reinterpret_cast<void *>(1));
    if (info) return info;
    if (!out) return GETT_ERR_STATE;
    features(a, prec, out);
    return 0;
}

static int64_t describe(int prec, int64_t order, int64_t tile, const Args &a, int64_t *out,
                        int64_t nout, bool tables) {
    const int info = validate(a, reinterpret_cast<void *>(1), reinterpret_cast<void *>(1),
                              reinterpret_cast<void *>(1));
    if (info) return info;
    if (prec < 0 || prec >= kNumPrec || prec == kFP8 || order < 0 || order >= kNumOrders ||
        tile < 0 || tile >= kNumTiles)
        return GETT_ERR_STATE;
    Canon c = canonicalise(a, (int)order, table_bn((int)prec, (int)tile));
    std::vector<int64_t> v;
    if (!tables) {
        v = {c.swapped, c.M, c.N, c.K, (int64_t)c.m.size(), (int64_t)c.n.size(),
             (int64_t)c.k.size(), c.aFastK, c.bFastK, c.boxX};
        for (auto *g : {&c.m, &c.n, &c.k})
            for (auto &x : *g) {
                v.push_back(x.ext);
                v.push_back(x.i0);
                v.push_back(x.i1);
            }
        int64_t r[4];
        operand_ranges(c, r[0], r[1], r[2], r[3]);
        v.insert(v.end(), r, r + 4);
    } else {
        if (c.empty) return 0;
        v.resize(2 * (c.M + c.N + c.K));
        int64_t *p = v.data();
        group_offsets(c.m, 0, c.M, p); p += c.M;
        group_offsets(c.m, 1, c.M, p); p += c.M;
        group_offsets(c.n, 0, c.N, p); p += c.N;
        group_offsets(c.n, 1, c.N, p); p += c.N;
        group_offsets(c.k, 0, c.K, p); p += c.K;
        group_offsets(c.k, 1, c.K, p);
    }
    if (out) {
        if ((int64_t)v.size() > nout) return GETT_ERR_STATE;
        std::copy(v.begin(), v.end(), out);
    }
    return (int64_t)v.size();
}

int64_t gett_plan_describe(int prec, int64_t order, int64_t tile, GETT_ARGS_DECL, int64_t *out,
                           int64_t nout) {
    return describe(prec, order, tile, GETT_ARGS_MAKE, out, nout, false);
}

int64_t gett_plan_tables(int prec, int64_t order, int64_t tile, GETT_ARGS_DECL, int64_t *out,
                         int64_t nout) {
    return describe(prec, order, tile, GETT_ARGS_MAKE, out, nout, true);
}

const char *gett_strerror(int code) {
    if (code == 0) return "success";
    if (code < 0) {
        static const char *names[] = {"RANKA", "EXTA", "INCA", "A", "RANKB", "EXTB", "INCB",
                                      "B", "CONTS", "CONTA", "CONTB", "PERM", "INCC", "C"};
        static thread_local char buf[64];
        if (code >= -14) {
            snprintf(buf, sizeof buf, "invalid argument %d (%s)", -code, names[-code - 1]);
            return buf;
        }
        return "invalid argument";
    }
    switch (code) {
    case GETT_ERR_HIP: {
        static thread_local char buf[128];
        snprintf(buf, sizeof buf, "HIP runtime error (last launch error: %s)",
                 last_hip_error_name());
        return buf;
    }
    case GETT_ERR_ALLOC: return "device allocation failed";
    case GETT_ERR_DEVICE: return "device is not gfx950 (MI355X)";
    case GETT_ERR_INTERNAL: return "internal planner limit";
    case GETT_ERR_STATE: return "invalid control call or state";
    case GETT_ERR_SCRATCH:
        return "problem too large for the allocation-free entry's scratch array";
    default: return "unknown error";
    }
}

int gett_finalize(void) {
    // Queued work may still read the tables, graphs and workspaces: wait for
    // the device before releasing them.
    int rc = 0;
    if (hipDeviceSynchronize() != hipSuccess) rc = GETT_ERR_HIP;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_graphs.clear();
        g_plans.clear();
        g_tables.clear();
        g_fp8.clear();
        g_tuned.clear();
        g_tuned_db.clear();
        g_tuned_db_read = false;   // a later tuning reads GETT_TUNE_DB again
    }
    unary_release();
    work_pools_trim();
    std::lock_guard<std::mutex> lk(g_pred_mu);
    g_pred.reset();
    return rc;
}

int gett_mlp_linear_fwd(const float *X, const float *W, const float *b, float *Y, int64_t batch,
                        int64_t d_in, int64_t d_out, int relu) {
    if (!X || !W || !b || !Y || batch < 1 || d_in < 1 || d_out < 1) return GETT_ERR_STATE;
    return launch_mlp_linear_fwd(X, W, b, Y, batch, d_in, d_out, relu, t_stream);
}
int gett_mlp_linear_bwd(const float *X, const float *W, const float *Y, const float *dY,
                        float *dX, float *dW, float *db, int64_t batch, int64_t d_in,
                        int64_t d_out, int relu) {
    if (!X || !W || !Y || !dY || !dW || !db || batch < 1 || d_in < 1 || d_out < 1)
        return GETT_ERR_STATE;
    return launch_mlp_linear_bwd(X, W, Y, dY, dX, dW, db, batch, d_in, d_out, relu, t_stream);
}
int gett_mlp_softmax_xent(const float *Z, const float *T, float *dZ, float *loss, int64_t batch,
                          int64_t nheads, const int64_t *head_sizes) {
    if (!Z || !T || !dZ || !loss || batch < 1 || nheads < 1 || nheads > 8 || !head_sizes)
        return GETT_ERR_STATE;
    int64_t total = 0;
    for (int64_t h = 0; h < nheads; ++h) {
        if (head_sizes[h] < 1 || head_sizes[h] > 64) return GETT_ERR_STATE;
        total += head_sizes[h];
    }
    return launch_mlp_xent(Z, T, dZ, loss, batch, total, nheads, head_sizes, t_stream);
}
int gett_mlp_adam(float *P, const float *G, float *m, float *v, int64_t n, float lr, float beta1,
                  float beta2, float eps, int64_t t) {
    if (!P || !G || !m || !v || n < 1 || t < 1) return GETT_ERR_STATE;
    return launch_mlp_adam(P, G, m, v, n, lr, beta1, beta2, eps, t, t_stream);
}

}  // extern "C"

// Host runtime of the compressed state-vector library: the C ABI of
// include/qcz.h on top of the kernels in qcz_kernels.hip.
//
// Device memory is one caller-owned pool, carved into
//   control block | chunk table | undo log | scan scratch | block levels |
//   reduction partials | staging | arena A | arena B.
// Compressed chunks are appended to the current arena; a chunk's previous
// stream stays where it was until the next compaction, so a gate can be
// undone by restoring table entries.  Compaction copies the live streams,
// in chunk order, into the other arena.
//
// Gates are launched in batches; each gate kernel's last workgroup logs the
// compressed size after the gate and raises a stop flag when the state no
// longer fits (budget of Sec. 3.7) or the arena is full.  Later gates of the
// batch then do nothing; the host rolls the stopped gate back, relaxes the
// level or compacts, and resumes from it.  This gives the per-gate decisions
// of Sec. 3.7 without a host round trip per gate.
#include "../../include/qcz.h"
#include "qcz_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

using namespace qcz;

namespace {

constexpr double kDelta[kLevels] = {0.0, 1e-5, 1e-4, 1e-3, 1e-2, 1e-1};
constexpr int kScratchChunks = 64;
constexpr int kMomGrid = 2048;
constexpr int kMaxGraphs = 8;
constexpr uint64_t kScanItems = 1024;
constexpr uint32_t kCacheIdleGates = 32;   // cached gates in a row without a hit that switch the cache off

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct GraphEntry {
    std::vector<uint8_t> key;
    hipGraphExec_t exec = nullptr;
};

struct Layout {
    size_t ds, table, undo, bsums, blevel, partials, wgp, scratch, cstats, feat, fn2, fsel, ckeys, cowner, crole,
        cparts, cjkey, rundesc, arena0, arena1, arena_bytes, end;
    uint64_t ctsize;   // block cache key slots (0: no cache)
};

// chunk statistics records held at once (blocks are processed in batches)
constexpr uint64_t kStatChunks = 65536;

int chunk_log2_for(int bl) { return bl < 10 ? bl : 10; }

Layout layout_for(int n, int bl, size_t pool_bytes, bool cache, bool fuse)
{
    const int cb = chunk_log2_for(bl);
    const int C = 2 << cb;
    const uint64_t nchunks = 1ull << (n - cb);
    const uint64_t nblocks = 1ull << (n - bl);
    Layout L{};
    size_t o = 0;
    L.ds = o; o = align256(o + sizeof(DevState));
    L.table = o; o = align256(o + 8 * nchunks);
    L.undo = o; o = align256(o + 8 * nchunks);
    L.bsums = o; o = align256(o + 8 * ((nchunks + kScanItems - 1) / kScanItems + 1));
    L.blevel = o; o = align256(o + nblocks);
    L.partials = o; o = align256(o + 8 * (size_t)std::max<uint64_t>(4 * kMomGrid, nchunks < (1u << 20) ? nchunks : 0));
    L.wgp = o; o = align256(o + sizeof(WgPart) * (size_t)kMaxGrid);
    const size_t slot = ((chunk_cap_bytes(C) + 3) & ~3u);
    L.scratch = o; o = align256(o + (size_t)kScratchChunks * (8 * (size_t)C + slot + 16) + 4096);
    L.cstats = o; o = align256(o + 8 * kChunkStats * (size_t)std::min<uint64_t>(nchunks, kStatChunks));
    L.feat = o; o = align256(o + 4 * kNIn * (size_t)nblocks);
    L.fn2 = o; o = align256(o + 8 * (size_t)nblocks);
    L.fsel = o; o = align256(o + (size_t)nblocks);
    // block cache: key slots for twice the jobs of a gate (at most nchunks / 2 jobs)
    L.ctsize = cache ? std::max<uint64_t>(64, nchunks) : 0;
    L.ckeys = o; o = align256(o + 8 * (size_t)L.ctsize);
    L.cowner = o; o = align256(o + 4 * (size_t)L.ctsize);
    L.crole = o; o = align256(o + 4 * (size_t)(cache ? std::max<uint64_t>(1, nchunks / 2) : 0));
    L.cparts = o; o = align256(o + (cache ? sizeof(WgPart) * (size_t)kCopyGrid : 0));
    L.cjkey = o; o = align256(o + 8 * (size_t)(cache ? std::max<uint64_t>(1, nchunks / 2) : 0));
    L.rundesc = o; o = align256(o + (fuse ? sizeof(GateDesc) * (size_t)kMaxBatch : 0));
    L.end = o;
    size_t rest = pool_bytes > o ? pool_bytes - o : 0;
    L.arena_bytes = (rest / 2) & ~(size_t)255;
    L.arena0 = o;
    L.arena1 = o + L.arena_bytes;
    return L;
}

}  // namespace

struct qcz_state {
    qcz_config cfg{};
    int n = 0, bl = 0, cb = 0, C = 0;
    uint64_t nchunks = 0, nblocks = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    uint8_t *pool = nullptr;
    size_t pool_bytes = 0;
    Layout lay{};
    DevState *ds = nullptr;
    uint64_t *table = nullptr, *undo = nullptr, *bsums = nullptr;
    WgPart *wgp = nullptr;
    uint8_t *blevel = nullptr;
    double *partials = nullptr;
    uint8_t *scratch = nullptr;
    uint32_t *arena[2] = {nullptr, nullptr};
    int cur = 0;
    int grid_max = 1024;
    int batch = 64;
    int chunk_waves = 4;
    // host mirror of the committed state
    int level = 0;
    uint64_t live = 0, bump = 0;          // bump: arena bytes in use (base + stripe fills)
    uint64_t base = 0, stripe_size = 0;   // arena stripes (see DevState)
    int nstripes = 1;
    uint64_t stripe_fill[kStripes] = {};
    uint64_t gates_applied = 0, lossy_steps = 0, min_c = 0, max_c = 0, compactions = 0;
    double flb = 1.0;
    double norm2 = 1.0;                   // squared norm of the stored state (per-block ledger)
    std::vector<uint8_t> block_levels;
    // learned per-block level selection, re-run every sel_period gates
    const float *sel_params = nullptr;
    double sel_beta = 0.0;
    uint64_t sel_period = 0, sel_since = 0;
    bool sel_fresh = false;
    bool broken = false;   // a gate run in ranges failed midway
    std::string err;
    std::vector<GraphEntry> graphs;
    DevState hds{};  // readback staging
    qcz_stats_t stats{};
    // launch-shape autotuner: candidate (waves, grid) shapes, measured round robin
    struct Cand { int waves, grid; double ms; uint64_t chunks; };
    std::vector<Cand> cands;
    int tune_next = 0;
    int tune_rounds = 0;
    bool tuning = false;
    std::vector<hipEvent_t> events;   // QCZ_FLAG_TIMING: start/stop per gate of a batch
    std::vector<int> timed;           // per gate of the batch: 1 if its fused kernel was timed
    // compressed block cache (QCZ_FLAG_CACHE)
    bool cache_on = false;
    uint64_t cache_key_mask = ~0ull;
    uint32_t cache_idle = 0;          // consecutive cached gates without a hit
    std::vector<uint8_t> cached;      // per gate of the batch: 1 if it ran through the cache
    // gate-layer fusion (QCZ_FLAG_FUSE): per gate of the batch, the first and
    // last gate of its fused run (-1: not in a run)
    std::vector<int> run_first, run_last;
    std::vector<GateDesc> run_desc;   // per batch position: the launch record of the run starting there
};

namespace {

qcz_status fail(qcz_state *s, qcz_status code, const std::string &msg)
{
    if (s) s->err = msg;
    return code;
}

#define HIPCHK(s, call)                                                                               \
    do {                                                                                              \
        hipError_t e_ = (call);                                                                       \
        if (e_ != hipSuccess) return fail((s), QCZ_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

DevPtrs ptrs(const qcz_state *s)
{
    DevPtrs P{};
    P.arena = s->arena[s->cur];
    P.out = P.arena;
    P.arena_words = s->lay.arena_bytes / 4;
    P.table = s->table;
    P.undo = s->undo;
    P.block_level = s->blevel;
    P.ds = s->ds;
    P.wgp = s->wgp;
    P.cb = s->cb;
    P.C = s->C;
    P.nchunks = s->nchunks;
    return P;
}

int popcount64(uint64_t x) { return __builtin_popcountll(x); }

// the state's encoder may take the entropy-coded body; its kernels decode it
int ent_state(const qcz_state *s) { return (s->cfg.flags & QCZ_FLAG_ENTROPY) ? 1 : 0; }
// the state's encoder stores values re parts first (Solution D)
int rsh_state(const qcz_state *s) { return (s->cfg.flags & QCZ_FLAG_RESHUFFLE) ? 1 : 0; }

// A stream header: mode, level, and the entropy bit (only where the state
// may hold entropy-coded streams, and never on a CONST2 stream).
bool header_ok(const qcz_state *s, uint32_t hdr, size_t len)
{
    const uint32_t mode = hdr & 3u, lev = (hdr >> 2) & 7u, ent = (hdr >> 5) & 1u, rsh = (hdr >> 6) & 1u;
    if ((hdr >> 7) != 0 || lev >= (uint32_t)kLevels || mode > M_SPARSE) return false;
    if (ent && (!ent_state(s) || mode == M_CONST2)) return false;
    if (rsh && mode == M_CONST2) return false;
    return mode != M_CONST2 || len == 20;
}

bool is_unit(double re, double im) { return re == 1.0 && im == 0.0; }

qcz_status check_gate(const qcz_state *s, const qcz_gate &g)
{
    const int n = s->n;
    const uint64_t all = (n >= 64) ? ~0ull : ((1ull << n) - 1);
    if (g.control_mask & ~all) return QCZ_E_INVAL;
    for (int k = 0; k < 8; ++k)
        if (!std::isfinite(g.m[k])) return QCZ_E_INVAL;
    switch (g.kind) {
    case K_U1:
    case K_DIAG1:
    case K_X:
        if ((int)g.target >= n) return QCZ_E_INVAL;
        if (g.control_mask & (1ull << g.target)) return QCZ_E_INVAL;
        return QCZ_OK;
    case K_DIAG2:
        if ((int)g.target >= n || (int)g.target2 >= n || g.target == g.target2) return QCZ_E_INVAL;
        if (g.control_mask & ((1ull << g.target) | (1ull << g.target2))) return QCZ_E_INVAL;
        return QCZ_OK;
    case K_MCZ:
        return g.control_mask ? QCZ_OK : QCZ_E_INVAL;
    default:
        return QCZ_E_INVAL;
    }
}

// Job builder: which chunks a gate touches (Sec. 3.3 index segments and
// control rules, at chunk granularity) as an enumeration over chunk bits.
GateDesc lower_gate(const qcz_state *s, const qcz_gate &g, int seq)
{
    GateDesc d{};
    d.kind = (int32_t)g.kind;
    d.q = (int32_t)g.target;
    d.q2 = (int32_t)g.target2;
    d.seq = seq;
    d.cm = g.control_mask;
    for (int k = 0; k < 8; ++k) d.m[k] = g.m[k];
    d.nchunk_bits = s->n - s->cb;
    d.per_block = s->cfg.mode == QCZ_MODE_PERBLOCK ? 1 : 0;
    d.block_shift = s->bl - s->cb;
    d.fixed_level = -1;
    d.entropy = ent_state(s);
    d.reshuffle = rsh_state(s);
    const uint64_t cm_hi = g.control_mask >> s->cb;
    const uint64_t cm_lo = g.control_mask & ((1ull << s->cb) - 1);
    if ((g.kind == K_U1 || g.kind == K_X) && (int)g.target >= s->cb) {
        d.pair_bit = 1ull << (g.target - s->cb);
        d.job_type = (g.kind == K_X && cm_lo == 0) ? J_PERMUTE : J_PAIR;
        d.fixed_mask = cm_hi | d.pair_bit;
        d.fixed_val = cm_hi;
        const int nfree = d.nchunk_bits - popcount64(d.fixed_mask);
        d.njobs = 1ull << nfree;
        d.nitems = d.job_type == J_PAIR ? 2 * d.njobs : d.njobs;
        return d;
    }
    d.job_type = J_SINGLE;
    d.fixed_mask = cm_hi;
    d.fixed_val = cm_hi;
    bool none = false;
    if (g.kind == K_DIAG1 || g.kind == K_DIAG2) {
        d.check_phase = 1;
        if (g.kind == K_DIAG1) {
            const bool u0 = is_unit(g.m[0], g.m[1]), u1 = is_unit(g.m[2], g.m[3]);
            if (u0 && u1) none = true;
            else if ((int)g.target >= s->cb && (u0 || u1)) {
                const uint64_t bit = 1ull << (g.target - s->cb);
                d.fixed_mask |= bit;
                if (u0) d.fixed_val |= bit;   // only the target=1 half has a non-trivial phase
            }
        } else if (is_unit(g.m[0], g.m[1]) && is_unit(g.m[2], g.m[3]) && is_unit(g.m[4], g.m[5]) &&
                   is_unit(g.m[6], g.m[7])) {
            none = true;
        }
    }
    const int nfree = d.nchunk_bits - popcount64(d.fixed_mask);
    d.nitems = none ? 0 : (1ull << nfree);
    d.njobs = (d.nitems + 1) / 2;
    return d;
}

int grid_for(const qcz_state *s, const GateDesc &d)
{
    if (d.job_type == J_PERMUTE) {
        uint64_t b = (d.njobs + kWG - 1) / kWG;
        return (int)std::max<uint64_t>(1, std::min<uint64_t>(b, 65535));
    }
    return (int)std::max<uint64_t>(1, std::min<uint64_t>(job_stop(d) - job_begin(d), (uint64_t)s->grid_max));
}

// enumerated chunk positions a launch covers (two per job)
uint64_t launch_items(const GateDesc &d)
{
    const uint64_t ipj = items_per_job(d);
    const uint64_t i0 = ipj * job_begin(d), i1 = std::min<uint64_t>(ipj * job_stop(d), d.nitems);
    return i1 > i0 ? i1 - i0 : 0;
}

qcz_status write_header(qcz_state *s)
{
    DevState h{};
    h.base = s->base;
    h.stripe_size = s->stripe_size;
    h.nstripes = (uint64_t)s->nstripes;
    h.live = s->live;
    h.arena_cap = s->lay.arena_bytes;
    h.budget = s->cfg.mode == QCZ_MODE_ADAPTIVE ? s->cfg.budget_bytes : 0;
    h.level = s->level;
    s->hds = h;
    HIPCHK(s, hipMemcpyAsync(s->ds, &s->hds, offsetof(DevState, stripe), hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));   // the staging struct is reused right after
    return QCZ_OK;
}

// Start fresh stripes right after the first `used` arena bytes.
qcz_status reset_stripes(qcz_state *s, uint64_t used)
{
    s->base = align256(used);
    const uint64_t cap = s->lay.arena_bytes;
    const uint64_t room = cap > s->base ? cap - s->base : 0;
    // as many stripes as leave room for 64 of the largest streams each
    uint64_t ns = room / (64ull * chunk_cap_bytes(s->C));
    s->nstripes = (int)std::max<uint64_t>(1, std::min<uint64_t>(ns, kStripes));
    s->stripe_size = (room / (uint64_t)s->nstripes) & ~(uint64_t)255;
    for (int k = 0; k < kStripes; ++k) s->stripe_fill[k] = 0;
    s->bump = s->base;
    for (int k = 0; k < kStripes; ++k) s->hds.stripe[k][0] = 0;
    HIPCHK(s, hipMemcpyAsync(&s->ds->stripe, &s->hds.stripe, sizeof(s->hds.stripe), hipMemcpyHostToDevice, s->stream));
    return write_header(s);
}

uint64_t max_stripe_fill(const qcz_state *s)
{
    uint64_t m = 0;
    for (int k = 0; k < s->nstripes; ++k) m = std::max(m, s->stripe_fill[k]);
    return m;
}

void clear_graphs(qcz_state *s)
{
    for (auto &g : s->graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    s->graphs.clear();
}

qcz_status compact(qcz_state *s)
{
    DevPtrs P = ptrs(s);
    const uint64_t nb = (s->nchunks + kScanItems - 1) / kScanItems;
    HIPCHK(s, launch_compact(P, s->arena[1 - s->cur], s->undo, s->bsums, nb, s->stream));
    uint64_t total = 0;
    HIPCHK(s, hipMemcpyAsync(&total, s->bsums + nb, 8, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    s->cur = 1 - s->cur;
    s->compactions += 1;
    // captured batches stay valid: they are keyed by the arena pointer and
    // read the stripe bases from the device header
    return reset_stripes(s, total);
}

// Expected bytes one stripe receives from gate `d`: every touched chunk gets a
// fresh stream, sized here at twice the current mean stream (plus slack) and
// never more than the largest stream; work-group w allocates in stripe
// w mod nstripes, so the fullest stripe serves ceil(grid / nstripes) groups.
uint64_t stripe_share(const qcz_state *s, const GateDesc &d)
{
    const uint64_t items = launch_items(d);
    if (d.job_type == J_PERMUTE || items == 0) return 0;
    const uint64_t mean = s->live / std::max<uint64_t>(1, s->nchunks);
    const uint64_t per = std::min<uint64_t>(2 * mean + 64, (uint64_t)chunk_cap_bytes(s->C) + 4);
    const uint64_t g = (uint64_t)grid_for(s, d);
    const uint64_t groups = (g + (uint64_t)s->nstripes - 1) / (uint64_t)s->nstripes;
    return (items * per * groups + g - 1) / g;
}

// gates that run through the block cache: fused jobs over a whole gate at a
// global level (per-block levels keep their own ledger per chunk)
bool cache_gate(const qcz_state *s, const GateDesc &d)
{
    return s->cache_on && d.job_type != J_PERMUTE && !d.per_block && d.job_end == 0 && d.njobs >= 2;
}

qcz_status launch_one(qcz_state *s, const GateDesc &d, bool timing)
{
    DevPtrs P = ptrs(s);
    if (cache_gate(s, d)) {
        // plan, leaders, follower copies, other followers: one gate over four launches, timed together
        CachePtrs cp{};
        cp.keys = (uint64_t *)(s->pool + s->lay.ckeys);
        cp.owner = (uint32_t *)(s->pool + s->lay.cowner);
        cp.role = (uint32_t *)(s->pool + s->lay.crole);
        cp.parts = (WgPart *)(s->pool + s->lay.cparts);
        cp.jkey = (uint64_t *)(s->pool + s->lay.cjkey);
        cp.tsize = 64;
        while (cp.tsize < 2 * d.njobs) cp.tsize *= 2;
        if (cp.tsize > s->lay.ctsize) return fail(s, QCZ_E_STATE, "block cache table too small");
        cp.key_mask = s->cache_key_mask;
        const int grid = std::min(grid_for(s, d), kMaxGrid / 2);
        if (timing) HIPCHK(s, hipEventRecord(s->events[2 * d.seq], s->stream));
        hipError_t e = launch_cache_plan(d, P, cp, s->stream);
        if (e == hipSuccess) e = launch_gate_list(d, P, cp, 1, grid, s->stream);
        if (e == hipSuccess) e = launch_cache_copy(d, P, cp, s->stream);
        if (e == hipSuccess) e = launch_gate_list(d, P, cp, 2, grid, s->stream);
        if (e != hipSuccess) return fail(s, QCZ_E_DEVICE, std::string("cached gate launch: ") + hipGetErrorString(e));
        if (timing) {
            HIPCHK(s, hipEventRecord(s->events[2 * d.seq + 1], s->stream));
            s->timed[(size_t)d.seq] = 1;
        }
        if ((size_t)d.seq < s->cached.size()) s->cached[(size_t)d.seq] = 1;
        return QCZ_OK;
    }
    const int grid = grid_for(s, d);
    const bool t = timing && d.job_type != J_PERMUTE;
    hipEvent_t t0 = t ? s->events[2 * d.seq] : nullptr, t1 = t ? s->events[2 * d.seq + 1] : nullptr;
    hipError_t e = d.job_type == J_PERMUTE ? launch_permute(d, P, grid, s->stream)
                                           : launch_gate(d, P, grid, s->stream, s->chunk_waves, t0, t1);
    if (e != hipSuccess) return fail(s, QCZ_E_DEVICE, std::string("gate launch: ") + hipGetErrorString(e));
    if (timing) s->timed[(size_t)d.seq] = t ? 1 : 0;
    return QCZ_OK;
}

// Gates a fused run may hold: every gate whose jobs lie inside single chunks
// (in-chunk targets of any kind, diagonal gates and multi-controlled Z on any
// qubits, with any controls), in modes whose level does not depend on the
// compressed size after each gate.  The run enumerates every chunk; each
// chunk takes, in order, the gates whose own enumeration and phases touch it,
// each followed by the truncation its re-encoding would apply, and is
// re-encoded once if any gate touched it.  Every such gate touches some
// chunk, so the ledger's per-gate lossy steps are those of the gates one by one.
bool fusable(const qcz_state *s, const GateDesc &d)
{
    return (s->cfg.flags & QCZ_FLAG_FUSE) && !s->cache_on && d.job_type == J_SINGLE && d.nitems > 0 &&
           !d.per_block && d.job_end == 0 && (s->cfg.mode == QCZ_MODE_FIXED || s->cfg.mode == QCZ_MODE_LOSSLESS);
}

// the launch record of a fused run: its first gate over every chunk
GateDesc run_launch(const qcz_state *s, const GateDesc &first)
{
    GateDesc r = first;
    r.fixed_mask = r.fixed_val = 0;
    r.check_phase = 0;
    r.act_mask = r.act_val = 0;
    r.nitems = s->nchunks;
    r.njobs = (s->nchunks + 1) / 2;
    return r;
}

// Gates a chunk-group run may hold: U1 / X whose target is a chunk-index bit
// (pair jobs, any controls), in the modes of fused runs, on 2048-double chunks
// without the entropy stage.  A run takes consecutive such gates on at most two
// distinct target bits; each job then holds the four chunks those bits join.
bool pairable(const qcz_state *s, const GateDesc &d)
{
    return (s->cfg.flags & QCZ_FLAG_FUSE) && (s->cfg.flags & QCZ_FLAG_GROUPS) && !s->cache_on && d.job_type == J_PAIR &&
           (d.kind == K_U1 || d.kind == K_X) &&
           !d.per_block && d.job_end == 0 && !ent_state(s) && s->C == kCMax && (s->n - s->cb) >= 2 &&
           (s->cfg.mode == QCZ_MODE_FIXED || s->cfg.mode == QCZ_MODE_LOSSLESS);
}

// Length of the run starting at descs[k] and its launch record: 0 (a lone
// gate), a fused run of single-chunk gates (kind 1, at least two gates) or a
// chunk-group run (kind 2, at least two gates).
size_t run_at(const qcz_state *s, const GateDesc *descs, size_t n, size_t k, GateDesc &launch, int &kind)
{
    kind = 0;
    size_t r = 0;
    while (k + r < n && r < (size_t)kMaxRun && fusable(s, descs[k + r])) ++r;
    if (r >= 2) {
        kind = 1;
        launch = run_launch(s, descs[k]);
        return r;
    }
    // target bits of the run: up to three distinct ones (eight-chunk groups)
    // when the state has that many chunk-index bits, else two
    const int maxbits = (s->n - s->cb) >= 3 ? 3 : 2;
    uint64_t bits[3] = {0, 0, 0};
    int nb = 0;
    r = 0;
    while (k + r < n && r < (size_t)kMaxRun && pairable(s, descs[k + r])) {
        const uint64_t pb = descs[k + r].pair_bit;
        bool known = false;
        for (int i = 0; i < nb; ++i) known = known || bits[i] == pb;
        if (!known) {
            if (nb == maxbits) break;
            bits[nb++] = pb;
        }
        ++r;
    }
    if (r < 2) return 0;
    if (nb == 1)   // one target bit: the lowest other chunk-index bit completes the groups
        for (int bit = 0; bit < s->n - s->cb; ++bit)
            if ((1ull << bit) != bits[0]) { bits[nb++] = 1ull << bit; break; }
    kind = 2;
    launch = descs[k];
    launch.job_type = J_GROUP;
    launch.pair_bit = bits[0];
    launch.pair_bit2 = bits[1];
    launch.pair_bit3 = nb == 3 ? bits[2] : 0;
    launch.fixed_mask = bits[0] | bits[1] | launch.pair_bit3;
    launch.fixed_val = 0;
    launch.check_phase = 0;
    launch.act_mask = launch.act_val = 0;
    launch.nitems = s->nchunks;
    launch.njobs = s->nchunks / items_per_job(launch);
    return r;
}

// chunk-group workgroups: four chunks (two workgroups per CU fit its LDS) or
// eight (one per CU); one resident round
int group_grid(const qcz_state *s, const GateDesc &d)
{
    const int g = std::max(1, d.pair_bit3 ? s->grid_max / 3 : s->grid_max * 2 / 3);
    return (int)std::max<uint64_t>(1, std::min<uint64_t>(d.njobs, (uint64_t)g));
}

// Number of leading gates of `descs` whose expected allocations fit in the
// room the fullest stripe has left.  Gates that the batch launches as one
// fused or chunk-group run allocate once per chunk for the whole run, so a
// run is counted once; a run that does not fit ends the count before it.
size_t gates_that_fit(const qcz_state *s, const std::vector<GateDesc> &descs)
{
    const uint64_t fill = max_stripe_fill(s);
    const uint64_t room = s->stripe_size > fill ? s->stripe_size - fill : 0;
    uint64_t acc = 0;
    size_t k = 0;
    while (k < descs.size()) {
        GateDesc launch;
        int kind = 0;
        size_t r = run_at(s, descs.data(), descs.size(), k, launch, kind);
        if (kind == 0) {
            r = 1;
            launch = descs[k];
        }
        acc += stripe_share(s, launch);
        if (acc > room) break;
        k += r;
    }
    return k;
}

// Leading gates of `descs` up to and including the first fused or chunk-group
// run.  A run re-encodes every chunk, and the arena estimates of a batch rest
// on the mean stream size before it: a run that turns a near-constant state
// dense (the first layer after Hadamards) would leave the next launch's
// estimate far too low, its appends would stop on a full arena, and the
// rollback, compaction and relaunch would cost more than a pass.  So a run
// ends its batch, and the next batch is planned from the sizes it left.
size_t through_first_run(const qcz_state *s, const std::vector<GateDesc> &descs)
{
    size_t k = 0;
    while (k < descs.size()) {
        GateDesc launch;
        int kind = 0;
        const size_t r = run_at(s, descs.data(), descs.size(), k, launch, kind);
        if (kind != 0) return k + r;
        k += 1;
    }
    return k;
}

qcz_status launch_batch(qcz_state *s, const std::vector<GateDesc> &descs)
{
    const bool timing = (s->cfg.flags & QCZ_FLAG_TIMING) != 0 || s->tuning;
    if (timing) {
        while (s->events.size() < 2 * descs.size()) {
            hipEvent_t ev;
            HIPCHK(s, hipEventCreate(&ev));
            s->events.push_back(ev);
        }
        s->timed.assign(descs.size(), 0);
    }
    s->cached.assign(descs.size(), 0);
    s->run_first.assign(descs.size(), -1);
    s->run_last.assign(descs.size(), -1);
    s->run_desc.assign(descs.size(), GateDesc{});
    if (timing || !(s->cfg.flags & QCZ_FLAG_GRAPH) || s->stream == nullptr) {
        GateDesc *dev_descs = (GateDesc *)(s->pool + s->lay.rundesc);
        bool uploaded = false;
        for (size_t k = 0; k < descs.size();) {
            GateDesc d;
            int kind = 0;
            const size_t r = run_at(s, descs.data(), descs.size(), k, d, kind);
            if (kind != 0) {
                if (!uploaded) {   // the batch's gate records, read by the fused runs
                    HIPCHK(s, hipMemcpyAsync(dev_descs, descs.data(), descs.size() * sizeof(GateDesc),
                                             hipMemcpyHostToDevice, s->stream));
                    uploaded = true;
                }
                hipEvent_t t0 = timing ? s->events[2 * d.seq] : nullptr, t1 = timing ? s->events[2 * d.seq + 1] : nullptr;
                hipError_t e = kind == 1
                                   ? launch_gate_run(d, ptrs(s), dev_descs + k, (int)r, grid_for(s, d), s->stream, t0, t1)
                                   : launch_group_run(d, ptrs(s), dev_descs + k, (int)r, group_grid(s, d), s->stream,
                                                      t0, t1);
                if (e != hipSuccess) return fail(s, QCZ_E_DEVICE, std::string("fused run launch: ") + hipGetErrorString(e));
                s->run_desc[k] = d;
                if (timing) s->timed[k] = 1;
                for (size_t j = k; j < k + r; ++j) {
                    s->run_first[j] = (int)k;
                    s->run_last[j] = (int)(k + r - 1);
                }
                k += r;
                continue;
            }
            qcz_status st = launch_one(s, descs[k], timing);
            if (st != QCZ_OK) return st;
            ++k;
        }
        if (uploaded) HIPCHK(s, hipStreamSynchronize(s->stream));   // the host records may change after return
        return QCZ_OK;
    }
    std::vector<uint8_t> key(descs.size() * sizeof(GateDesc) + sizeof(DevPtrs) + 1);
    DevPtrs P = ptrs(s);
    memcpy(key.data(), &P, sizeof(P));
    key.back() = s->cache_on ? 1 : 0;   // the launches of a cached gate differ
    if (!descs.empty()) memcpy(key.data() + sizeof(P), descs.data(), descs.size() * sizeof(GateDesc));
    for (auto &g : s->graphs) {
        if (g.key == key) {
            HIPCHK(s, hipGraphLaunch(g.exec, s->stream));
            return QCZ_OK;
        }
    }
    hipGraph_t graph = nullptr;
    HIPCHK(s, hipStreamBeginCapture(s->stream, hipStreamCaptureModeRelaxed));
    qcz_status st = QCZ_OK;
    for (const auto &d : descs) {
        st = launch_one(s, d, false);
        if (st != QCZ_OK) break;
    }
    hipError_t e = hipStreamEndCapture(s->stream, &graph);
    if (st != QCZ_OK) return st;
    if (e != hipSuccess) return fail(s, QCZ_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(s, QCZ_E_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
    if ((int)s->graphs.size() >= kMaxGraphs) {
        (void)hipGraphExecDestroy(s->graphs.front().exec);
        s->graphs.erase(s->graphs.begin());
    }
    GraphEntry ge;
    ge.key = std::move(key);
    ge.exec = exec;
    s->graphs.push_back(std::move(ge));
    HIPCHK(s, hipGraphLaunch(exec, s->stream));
    return QCZ_OK;
}

// kind: 0 a one-gate pass, 1 a fused run, 2 a chunk-group run (per-kind counters)
void commit_gate(qcz_state *s, const GateLog &lg, const GateDesc &d, int k, bool tbl = true, int kind = 0)
{
    s->live = lg.live;
    s->bump = lg.bump;
    s->gates_applied += 1;
    qcz_stats_t &S = s->stats;
    if (d.job_type == J_PERMUTE) {
        S.permute_launches += 1;
    } else {
        S.gate_launches += 1;
        S.chunks_reencoded += lg.reenc;
        S.amps_touched += lg.reenc * (uint64_t)(s->C / 2);
        S.bytes_read += lg.rd;
        S.bytes_written += lg.wr;
        if (tbl) S.table_bytes += 24 * lg.reenc;
        S.kind_bytes[kind] += lg.rd + lg.wr + (tbl ? 24 * lg.reenc : 0);
        if (k < (int)s->cached.size() && s->cached[(size_t)k]) {
            // Sec. 3.4: the cache is switched off when it keeps missing
            S.cache_gates += 1;
            S.cache_hits += lg.hits;
            s->cache_idle = lg.hits ? 0 : s->cache_idle + 1;
            if (s->cache_idle >= kCacheIdleGates) s->cache_on = false;
        }
        if (k < (int)s->timed.size() && s->timed[(size_t)k]) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, s->events[2 * (size_t)k], s->events[2 * (size_t)k + 1]) == hipSuccess) {
                if (s->cfg.flags & QCZ_FLAG_TIMING) {
                    S.timed_launches += 1;
                    S.gate_kernel_ms += ms;
                    S.kind_launches[kind] += 1;
                    S.kind_kernel_ms[kind] += ms;
                }
                if (s->tuning) {
                    auto &c = s->cands[(size_t)s->tune_next];
                    c.ms += ms;
                    c.chunks += lg.reenc;
                }
            }
        }
    }
    if (s->cfg.mode == QCZ_MODE_PERBLOCK) {
        // Sec. 3.8 with a bound that varies by chunk: the step keeps the
        // fidelity at least 1 - wd / |state|^2, wd = sum over re-encoded
        // chunks of delta(level) * |chunk before truncation|^2
        if (lg.wd > 0.0) {
            s->flb *= (1.0 - lg.wd / s->norm2);
            s->lossy_steps += 1;
        }
        s->norm2 -= lg.lost;
    } else if (lg.reenc > 0 && kDelta[s->level] > 0.0) {
        s->flb *= (1.0 - kDelta[s->level]);   // Sec. 3.8, Eq. (11)
        s->lossy_steps += 1;
    }
    s->min_c = std::min(s->min_c, s->live);
    s->max_c = std::max(s->max_c, s->live);
}

// Commit gate k of a batch from the device log.  A gate of a fused run takes
// the run's log (one pass re-encoded every chunk once per gate of the run, in
// effect): the chunks and live bytes after the run, its stream bytes and
// table traffic counted once, on the run's last gate.
void commit_logged(qcz_state *s, const DevState &h, const GateDesc &d, int k)
{
    const int f = k < (int)s->run_first.size() ? s->run_first[(size_t)k] : -1;
    if (f < 0) {
        commit_gate(s, h.log[k], d, k);
        return;
    }
    GateLog lg = h.log[f];
    const bool last = k == s->run_last[(size_t)k];
    if (!last) lg.rd = lg.wr = 0;
    commit_gate(s, lg, d, k, last, s->run_desc[(size_t)f].job_type == J_GROUP ? 2 : 1);
}

// Move the autotuner to its next candidate; after kTuneRounds passes over
// the candidates keep the one with the least kernel time per chunk.
constexpr int kTuneRounds = 2;

void tune_step(qcz_state *s)
{
    if (!s->tuning) return;
    s->tune_next += 1;
    if (s->tune_next < (int)s->cands.size()) return;
    s->tune_next = 0;
    s->tune_rounds += 1;
    if (s->tune_rounds < kTuneRounds) return;
    int best = -1;
    double best_cost = 0.0;
    for (size_t i = 0; i < s->cands.size(); ++i) {
        const auto &c = s->cands[i];
        if (c.chunks == 0) continue;
        const double cost = c.ms / (double)c.chunks;
        if (best < 0 || cost < best_cost) { best = (int)i; best_cost = cost; }
    }
    if (best >= 0) {
        s->chunk_waves = s->cands[(size_t)best].waves;
        s->grid_max = s->cands[(size_t)best].grid;
    }
    s->tuning = false;
    clear_graphs(s);
}

qcz_status single_kernel_chunks(qcz_state *s, GateDesc &d, uint64_t nitems, uint64_t first)
{
    d = GateDesc{};
    d.job_type = J_SINGLE;
    d.nitems = nitems;
    d.njobs = (nitems + 1) / 2;
    d.fixed_level = -1;
    d.entropy = ent_state(s);
    d.reshuffle = rsh_state(s);
    int bits = 0;
    while ((1ull << bits) < nitems) ++bits;
    d.nchunk_bits = bits;
    (void)first;
    return QCZ_OK;
}

// Statistics of every block: 16 float features into X (device, nblocks x 16)
// and the squared norm of each block into n2 (device, may be null).
qcz_status block_stats(qcz_state *s, double beta, uint64_t mask, float *X, double *n2)
{
    const int shift = s->bl - s->cb;
    const uint64_t cpb = 1ull << shift;
    if (cpb > kStatChunks) return fail(s, QCZ_E_INVAL, "blocks of more than 65536 chunks");
    FeatCtx ctx{};
    ctx.f12 = beta > 0.0 ? std::max(std::log10(beta), -20.0) / 5.0 : -4.0;
    ctx.f13 = std::log2(std::ldexp(1.0, s->n + 4) / (double)s->live) / 16.0;
    ctx.f14 = std::log2((double)s->nblocks) / 16.0;
    ctx.f15 = (double)__builtin_popcountll(mask) / 16.0;
    ctx.cpb = (int32_t)cpb;
    ctx.block_log2 = s->bl;
    ctx.nblocks = s->nblocks;
    double *cs = (double *)(s->pool + s->lay.cstats);
    const uint64_t per = std::max<uint64_t>(1, kStatChunks / cpb);   // blocks per batch
    for (uint64_t b0 = 0; b0 < s->nblocks; b0 += per) {
        const uint64_t nb = std::min<uint64_t>(per, s->nblocks - b0);
        GateDesc d{};
        single_kernel_chunks(s, d, nb << shift, 0);
        d.block_shift = shift;
        IOPtrs io{};
        io.first = b0 << shift;
        io.cstats = cs;
        const int grid = (int)std::max<uint64_t>(1, std::min<uint64_t>(d.njobs, (uint64_t)s->grid_max));
        HIPCHK(s, launch_chunk_stats(d, ptrs(s), io, grid, s->stream));
        HIPCHK(s, launch_block_features(cs, s->blevel + b0, ctx, nb, X + b0 * kNIn, n2 ? n2 + b0 : nullptr,
                                        s->stream));
    }
    return QCZ_OK;
}

// Run one gate whose new streams do not fit next to the live ones: launch
// its jobs in ranges, each committed before the next (the streams a range
// replaced become garbage that compaction reclaims).  Each range takes as
// many jobs as the free room of the fullest stripe holds at the current
// bytes-per-chunk estimate (twice the mean stream at first, then 1.25 times
// what the previous range wrote per chunk, the largest stream after a stop);
// the arena is compacted when the room holds less than a sixteenth of the
// gate.  A range stopped by a full arena is undone, the arena compacted and
// the range retried at half the size per repeated stop (a single job that
// still does not fit is QCZ_E_NOMEM).  Only for modes without a compressed-size budget: a
// budget overflow must undo the whole gate, which needs all of its old
// streams.  The gate counts once in the ledger and the statistics; its
// launches are not event-timed.
bool ranges_allowed(const qcz_state *s)
{
    return (s->cfg.flags & QCZ_FLAG_RANGES) && s->cfg.mode != QCZ_MODE_ADAPTIVE;
}

qcz_status apply_in_ranges(qcz_state *s, const GateDesc &d)
{
    const uint64_t nj = d.njobs;
    const uint64_t cap = (uint64_t)chunk_cap_bytes(s->C) + 4;
    uint64_t per = std::min<uint64_t>(2 * (s->live / std::max<uint64_t>(1, s->nchunks)) + 64, cap);
    uint64_t j = 0;
    int stops_here = 0;
    GateLog tot{};
    auto room = [&]() {
        const uint64_t fill = max_stripe_fill(s);
        return s->stripe_size > fill ? s->stripe_size - fill : 0;
    };
    // jobs (two chunks each) whose new streams fit in `r` bytes of the fullest stripe
    auto jobs_fitting = [&](uint64_t r) {
        const uint64_t gm = (uint64_t)std::max(1, s->grid_max), ns = (uint64_t)std::max(1, s->nstripes);
        const uint64_t groups = (gm + ns - 1) / ns;
        const uint64_t big = r * gm / (2 * per * groups);
        if (big >= gm) return big;
        return std::min<uint64_t>(gm - 1, ns * (r / (2 * per)));
    };
    while (j < nj) {
        const uint64_t left = nj - j;
        uint64_t L = std::min<uint64_t>(left, jobs_fitting(room()));
        if (L < std::min<uint64_t>(left, std::max<uint64_t>(1, nj / 16)) && s->bump > s->base) {
            qcz_status st = compact(s);
            if (st != QCZ_OK) return st;
            L = std::min<uint64_t>(left, jobs_fitting(room()));
        }
        L >>= std::min(stops_here, 40);   // repeated stops: smaller ranges
        if (L == 0) L = 1;                 // the device check decides
        GateDesc r = d;
        r.seq = 0;
        r.job0 = j;
        r.job_end = j + L;
        const uint64_t live0 = s->live, bump0 = s->bump;
        // with QCZ_FLAG_TIMING each range launch is timed like a whole gate
        const bool timing = (s->cfg.flags & QCZ_FLAG_TIMING) != 0;
        if (timing) {
            while (s->events.size() < 2) {
                hipEvent_t ev;
                HIPCHK(s, hipEventCreate(&ev));
                s->events.push_back(ev);
            }
            s->timed.assign(1, 0);
        }
        qcz_status st = launch_one(s, r, timing);
        if (st != QCZ_OK) return st;
        HIPCHK(s, hipMemcpyAsync(&s->hds, s->ds, offsetof(DevState, log) + sizeof(GateLog), hipMemcpyDeviceToHost,
                                 s->stream));
        HIPCHK(s, hipStreamSynchronize(s->stream));
        if (timing && s->timed[0]) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, s->events[0], s->events[1]) == hipSuccess) {
                s->stats.timed_launches += 1;
                s->stats.gate_kernel_ms += ms;
                s->stats.range_launches += 1;
                s->stats.kind_launches[0] += 1;
                s->stats.kind_kernel_ms[0] += ms;
            }
        }
        const DevState &h = s->hds;
        for (int k = 0; k < kStripes; ++k) s->stripe_fill[k] = h.stripe[k][0];
        if (!h.stop) {
            const GateLog &lg = h.log[0];
            s->live = lg.live;
            s->bump = lg.bump;
            tot.reenc += lg.reenc;
            tot.rd += lg.rd;
            tot.wr += lg.wr;
            tot.wd += lg.wd;
            tot.lost += lg.lost;
            if (lg.reenc) per = std::min<uint64_t>(cap, std::max<uint64_t>(64, lg.wr / lg.reenc * 5 / 4));
            j = r.job_end;
            stops_here = 0;
            continue;
        }
        const int reason = h.stop_reason;
        s->stats.stops += 1;
        DevPtrs P = ptrs(s);
        const int rg = (int)std::max<uint64_t>(1, std::min<uint64_t>((launch_items(r) + kWG - 1) / kWG, 65535));
        HIPCHK(s, launch_rollback(r, P, rg, s->stream));
        s->live = live0;
        s->bump = bump0;
        st = write_header(s);
        if (st != QCZ_OK) return st;
        if (reason != STOP_ARENA) {
            (void)hipStreamSynchronize(s->stream);
            return fail(s, QCZ_E_FORMAT, "a chunk table entry points outside the arena");
        }
        if (L == 1 && stops_here > 0) {
            if (j == 0) return fail(s, QCZ_E_NOMEM, "arena too small for one job of a gate");
            s->broken = true;   // earlier ranges of this gate are committed and cannot be undone
            return fail(s, QCZ_E_NOMEM, "arena ran out midway through a gate run in ranges: the state is invalid");
        }
        per = cap;                       // size the next attempt for the largest streams
        stops_here += 1;
        st = compact(s);
        if (st != QCZ_OK) return st;
    }
    tot.live = s->live;
    tot.bump = s->bump;
    s->stats.range_gates += 1;
    s->cached.clear();   // job ranges never run through the block cache
    s->timed.clear();    // (the ranges' kernel time is already counted)
    commit_gate(s, tot, d, 0);
    return QCZ_OK;
}

// Sweep: a gate (or a fused run of in-chunk gates) whose new streams do not
// fit beside the live ones runs as one launch that writes every chunk into
// the other arena, the chunks it leaves unchanged copied there as they are.
// The current arena is only read, so a stop (budget or full arena) is undone
// by restoring the table entries, and a success swaps the arenas' roles: the
// compaction comes with the gate, where job ranges would compact several
// times per gate.  The sweep's enumeration covers every chunk; the control
// bits the plain enumeration holds fixed become the act mask.
bool sweepable(const qcz_state *s, const GateDesc &d)
{
    (void)s;
    return d.job_type != J_PERMUTE && d.nitems > 0 && d.job_end == 0;
}

GateDesc sweep_desc(const GateDesc &d)
{
    GateDesc r = d;
    r.sweep = 1;
    r.act_mask = d.fixed_mask & ~d.pair_bit;
    r.act_val = d.fixed_val & r.act_mask;
    r.fixed_mask = d.fixed_mask & d.pair_bit;   // 0 for jobs inside chunks
    r.fixed_val = 0;
    const int nfree = d.nchunk_bits - popcount64(r.fixed_mask);
    if (d.job_type == J_PAIR) {
        r.njobs = 1ull << nfree;
        r.nitems = 2 * r.njobs;
    } else {
        r.nitems = 1ull << nfree;
        r.njobs = (r.nitems + 1) / 2;
    }
    return r;
}

// the state, a sixteenth for growth and the 16-byte allocation units, in an
// empty arena less a thirty-second for unevenly filled stripes
bool sweep_may_fit(const qcz_state *s)
{
    const uint64_t need = s->live + s->live / 16 + 16 * s->nchunks;
    return need <= s->lay.arena_bytes - s->lay.arena_bytes / 32;
}

// Run descs[0 .. r) as a sweep (kind 1: a fused run, kind 2: a chunk-group
// run, launched from `launch`).  *reason: STOP_NONE when committed, else why
// the device stopped it (the state is then unchanged).
qcz_status apply_sweep(qcz_state *s, const GateDesc *descs, size_t r, int kind, const GateDesc &launch, int *reason)
{
    *reason = STOP_NONE;
    const uint64_t base0 = s->base, ssize0 = s->stripe_size, live0 = s->live, bump0 = s->bump;
    const int ns0 = s->nstripes;
    uint64_t fill0[kStripes];
    for (int k = 0; k < kStripes; ++k) fill0[k] = s->stripe_fill[k];
    const int other = 1 - s->cur;
    // stripes over the whole other arena (the header describes the arena written to)
    qcz_status st = reset_stripes(s, 0);
    if (st != QCZ_OK) return st;
    GateDesc d = launch;
    if (kind == 2) d.sweep = 1;   // (its enumeration covers every chunk already)
    else d = sweep_desc(launch);
    d.seq = 0;
    DevPtrs P = ptrs(s);
    P.out = s->arena[other];
    const bool timing = (s->cfg.flags & QCZ_FLAG_TIMING) != 0;
    if (timing)
        while (s->events.size() < 2) {
            hipEvent_t ev;
            HIPCHK(s, hipEventCreate(&ev));
            s->events.push_back(ev);
        }
    hipEvent_t t0 = timing ? s->events[0] : nullptr, t1 = timing ? s->events[1] : nullptr;
    const int grid = kind == 2 ? group_grid(s, d) : grid_for(s, d);
    hipError_t e;
    if (kind != 0) {
        GateDesc *dev_descs = (GateDesc *)(s->pool + s->lay.rundesc);
        HIPCHK(s, hipMemcpyAsync(dev_descs, descs, r * sizeof(GateDesc), hipMemcpyHostToDevice, s->stream));
        e = kind == 1 ? launch_gate_run(d, P, dev_descs, (int)r, grid, s->stream, t0, t1)
                      : launch_group_run(d, P, dev_descs, (int)r, grid, s->stream, t0, t1);
    } else {
        e = launch_gate(d, P, grid, s->stream, s->chunk_waves, t0, t1);
    }
    if (e != hipSuccess) return fail(s, QCZ_E_DEVICE, std::string("sweep launch: ") + hipGetErrorString(e));
    HIPCHK(s, hipMemcpyAsync(&s->hds, s->ds, offsetof(DevState, log) + sizeof(GateLog), hipMemcpyDeviceToHost,
                             s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    const DevState &h = s->hds;
    if (!h.stop) {
        s->cur = other;
        for (int k = 0; k < kStripes; ++k) s->stripe_fill[k] = h.stripe[k][0];
        if (timing) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, s->events[0], s->events[1]) == hipSuccess) {
                s->stats.timed_launches += 1;
                s->stats.gate_kernel_ms += ms;
                s->stats.kind_launches[kind] += 1;
                s->stats.kind_kernel_ms[kind] += ms;
            }
        }
        // a fused run commits like one of launch_batch: every gate takes the
        // run's log, its stream bytes and table traffic counted on the last
        s->timed.clear();
        s->cached.clear();
        for (size_t k = 0; k < r; ++k) {
            GateLog lg = h.log[0];
            if (k + 1 < r) lg.rd = lg.wr = 0;
            commit_gate(s, lg, descs[k], (int)k, k + 1 == r, kind);
        }
        s->stats.sweep_gates += r;
        return QCZ_OK;
    }
    *reason = h.stop_reason;
    s->stats.stops += 1;
    const int rg = (int)std::max<uint64_t>(1, std::min<uint64_t>((launch_items(d) + kWG - 1) / kWG, 65535));
    HIPCHK(s, launch_rollback(d, P, rg, s->stream));
    // the current arena's allocator as it was
    s->base = base0;
    s->stripe_size = ssize0;
    s->nstripes = ns0;
    s->live = live0;
    s->bump = bump0;
    for (int k = 0; k < kStripes; ++k) {
        s->stripe_fill[k] = fill0[k];
        s->hds.stripe[k][0] = fill0[k];
    }
    HIPCHK(s, hipMemcpyAsync(&s->ds->stripe, &s->hds.stripe, sizeof(s->hds.stripe), hipMemcpyHostToDevice, s->stream));
    return write_header(s);
}

// Blocks grouped by coset id b & ~mask: cosets in increasing id, members in
// block order, and the weight of each coset summed in block order.
struct Cosets {
    std::vector<uint64_t> ids;      // distinct coset ids, increasing
    std::vector<double> W;          // per coset
    std::vector<uint64_t> start;    // members of coset k: mem[start[k] .. start[k+1])
    std::vector<uint64_t> mem;
};

Cosets make_cosets(const double *w, uint64_t nb, uint64_t mask)
{
    Cosets c;
    std::vector<int64_t> slot(nb, -1);
    for (uint64_t b = 0; b < nb; ++b) {
        const uint64_t id = b & ~mask;
        if (slot[id] < 0) slot[id] = 0;
    }
    for (uint64_t id = 0; id < nb; ++id)
        if (slot[id] >= 0) { slot[id] = (int64_t)c.ids.size(); c.ids.push_back(id); }
    const size_t nc = c.ids.size();
    c.W.assign(nc, 0.0);
    std::vector<uint64_t> cnt(nc + 1, 0);
    for (uint64_t b = 0; b < nb; ++b) {
        const size_t k = (size_t)slot[b & ~mask];
        c.W[k] += w[b];
        cnt[k + 1] += 1;
    }
    c.start.assign(nc + 1, 0);
    for (size_t k = 0; k < nc; ++k) c.start[k + 1] = c.start[k] + cnt[k + 1];
    c.mem.assign(nb, 0);
    std::vector<uint64_t> fill(c.start.begin(), c.start.end() - 1);
    for (uint64_t b = 0; b < nb; ++b) c.mem[fill[(size_t)slot[b & ~mask]]++] = b;
    return c;
}

// While sum over cosets of W_c * delta(max level in c) exceeds
// beta * (1 + 2^-20), lower by one every block at the max level of the coset
// with the largest W_c * delta(max level) (lowest coset id on ties).  The
// running sum is confirmed by an in-order sum whenever it is near the limit,
// so the stopping point is that of the in-order sum.
void project(const double *w, uint64_t nb, double beta, uint64_t mask, uint8_t *L)
{
    const double lim = beta * (1.0 + std::ldexp(1.0, -20));
    const Cosets cs = make_cosets(w, nb, mask);
    const size_t nc = cs.ids.size();
    std::vector<int> top(nc, 0);
    for (size_t k = 0; k < nc; ++k)
        for (uint64_t i = cs.start[k]; i < cs.start[k + 1]; ++i) top[k] = std::max(top[k], (int)L[cs.mem[i]]);
    auto exact = [&]() {
        double t = 0.0;
        for (size_t k = 0; k < nc; ++k) t += cs.W[k] * kDelta[top[k]];
        return t;
    };
    double run = exact();
    if (run <= lim) return;
    // max-heap on (W_c * delta(top_c), -k)
    std::vector<std::pair<double, int64_t>> heap;
    for (size_t k = 0; k < nc; ++k)
        if (top[k] > 0 && cs.W[k] * kDelta[top[k]] > 0.0) heap.push_back({cs.W[k] * kDelta[top[k]], -(int64_t)k});
    std::make_heap(heap.begin(), heap.end());
    while (!heap.empty()) {
        std::pop_heap(heap.begin(), heap.end());
        const auto h = heap.back();
        heap.pop_back();
        const size_t k = (size_t)(-h.second);
        for (uint64_t i = cs.start[k]; i < cs.start[k + 1]; ++i)
            if (L[cs.mem[i]] == top[k]) L[cs.mem[i]] -= 1;
        run -= h.first;
        top[k] -= 1;
        const double v = cs.W[k] * kDelta[top[k]];
        run += v;
        if (top[k] > 0 && v > 0.0) {
            heap.push_back({v, -(int64_t)k});
            std::push_heap(heap.begin(), heap.end());
        }
        if (run <= lim * (1.0 + 1e-9) && exact() <= lim) return;
    }
}

// The loosest level whose delta is at most beta (0, lossless, for beta < 1e-5).
uint8_t rule_level(double beta)
{
    uint8_t r = 0;
    for (int lev = 1; lev < kLevels; ++lev)
        if (kDelta[lev] <= beta) r = (uint8_t)lev;
    return r;
}

// Block-index bits that the gates may flip: targets of U1 / X gates on
// block-index qubits.  Weight only moves inside cosets of these bits.
uint64_t mixing_mask(const qcz_state *s, const qcz_gate *g, size_t n)
{
    uint64_t m = 0;
    for (size_t k = 0; k < n; ++k)
        if ((g[k].kind == (uint32_t)K_U1 || g[k].kind == (uint32_t)K_X) && (int)g[k].target >= s->bl)
            m |= 1ull << (g[k].target - (uint32_t)s->bl);
    return m;
}

qcz_status select_levels(qcz_state *s, const float *params, double beta, uint64_t mask, uint8_t *out_levels)
{
    if (s->cfg.mode != QCZ_MODE_PERBLOCK) return fail(s, QCZ_E_STATE, "level selection needs QCZ_MODE_PERBLOCK");
    float *X = (float *)(s->pool + s->lay.feat);
    double *n2 = (double *)(s->pool + s->lay.fn2);
    uint8_t *sel = s->pool + s->lay.fsel;
    qcz_status st = block_stats(s, beta, mask, X, n2);
    if (st != QCZ_OK) return st;
    HIPCHK(s, launch_mlp_forward(params, X, s->nblocks, nullptr, sel, s->stream));
    std::vector<uint8_t> L(s->nblocks);
    std::vector<double> w(s->nblocks);
    HIPCHK(s, hipMemcpyAsync(L.data(), sel, s->nblocks, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipMemcpyAsync(w.data(), n2, 8 * s->nblocks, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    double tot = 0.0;
    for (double x : w) tot += x;
    for (double &x : w) x = tot > 0.0 ? x / tot : 0.0;
    // Floor at the rule's level (the loosest level with delta <= beta): one
    // bound for every block already meets the budget, so a tighter level
    // only costs bytes; the projection may still lower blocks below it.
    const uint8_t rule = rule_level(beta);
    for (auto &l : L) l = std::max(l, rule);
    project(w.data(), s->nblocks, beta, mask, L.data());
    s->block_levels = L;
    HIPCHK(s, hipMemcpyAsync(s->blevel, s->block_levels.data(), s->nblocks, hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    if (out_levels) memcpy(out_levels, L.data(), s->nblocks);
    return QCZ_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

size_t qcz_chunk_cap(uint32_t C)
{
    if (C < 4 || (C & (C - 1))) return 0;
    return chunk_cap_bytes((int)C);
}

size_t qcz_pool_bytes_min(const qcz_config *cfg)
{
    if (!cfg || cfg->n_qubits < 6 || cfg->n_qubits > 40 || cfg->block_log2 < 6 || cfg->block_log2 > cfg->n_qubits)
        return 0;
    Layout L = layout_for((int)cfg->n_qubits, (int)cfg->block_log2, 0, (cfg->flags & QCZ_FLAG_CACHE) != 0,
                          (cfg->flags & QCZ_FLAG_FUSE) != 0);
    const int cb = chunk_log2_for((int)cfg->block_log2);
    const uint64_t nchunks = 1ull << (cfg->n_qubits - cb);
    // two arenas, each holding the initial streams with room to spare
    const size_t arena = align256((size_t)(64u << 10) + 64 * (size_t)nchunks);
    return L.end + 2 * arena;
}

qcz_status qcz_create(const qcz_config *cfg, void *dev_pool, size_t pool_bytes, void *hip_stream, qcz_state **out)
{
    if (!cfg || !out || !dev_pool) return QCZ_E_INVAL;
    *out = nullptr;
    if (cfg->n_qubits < 6 || cfg->n_qubits > 40 || cfg->block_log2 < 6 || cfg->block_log2 > cfg->n_qubits)
        return QCZ_E_INVAL;
    if (cfg->mode < QCZ_MODE_LOSSLESS || cfg->mode > QCZ_MODE_PERBLOCK) return QCZ_E_INVAL;
    if (cfg->level < 0 || cfg->level >= kLevels || cfg->batch > (uint32_t)kMaxBatch) return QCZ_E_INVAL;
    if (cfg->chunk_waves != 0 && cfg->chunk_waves != 2 && cfg->chunk_waves != 4 && cfg->chunk_waves != 8)
        return QCZ_E_INVAL;
    if (((uintptr_t)dev_pool & 255) != 0) return QCZ_E_INVAL;
    if ((cfg->flags & (QCZ_FLAG_CACHE | QCZ_FLAG_FUSE)) && (cfg->flags & QCZ_FLAG_AUTOTUNE)) return QCZ_E_INVAL;
    if ((cfg->flags & QCZ_FLAG_ENTROPY) &&
        (cfg->block_log2 < 10 || (cfg->flags & (QCZ_FLAG_CACHE | QCZ_FLAG_AUTOTUNE)) ||
         (cfg->chunk_waves != 0 && cfg->chunk_waves != 2)))
        return QCZ_E_INVAL;
    if (pool_bytes < qcz_pool_bytes_min(cfg)) return QCZ_E_NOMEM;

    qcz_state *s = new qcz_state();
    s->cfg = *cfg;
    s->n = (int)cfg->n_qubits;
    s->bl = (int)cfg->block_log2;
    s->cb = chunk_log2_for(s->bl);
    s->C = 2 << s->cb;
    s->nchunks = 1ull << (s->n - s->cb);
    s->nblocks = 1ull << (s->n - s->bl);
    s->pool = (uint8_t *)dev_pool;
    s->pool_bytes = pool_bytes;
    s->lay = layout_for(s->n, s->bl, pool_bytes, (cfg->flags & QCZ_FLAG_CACHE) != 0, (cfg->flags & QCZ_FLAG_FUSE) != 0);
    s->ds = (DevState *)(s->pool + s->lay.ds);
    s->table = (uint64_t *)(s->pool + s->lay.table);
    s->undo = (uint64_t *)(s->pool + s->lay.undo);
    s->bsums = (uint64_t *)(s->pool + s->lay.bsums);
    s->blevel = s->pool + s->lay.blevel;
    s->partials = (double *)(s->pool + s->lay.partials);
    s->wgp = (WgPart *)(s->pool + s->lay.wgp);
    s->scratch = s->pool + s->lay.scratch;
    s->arena[0] = (uint32_t *)(s->pool + s->lay.arena0);
    s->arena[1] = (uint32_t *)(s->pool + s->lay.arena1);
    s->batch = cfg->batch ? (int)cfg->batch : 64;
    s->chunk_waves = cfg->chunk_waves ? (int)cfg->chunk_waves : 2;
    while (s->chunk_waves > 2 && s->C < 64 * s->chunk_waves) s->chunk_waves /= 2;   // at least one value per thread
    s->level = cfg->mode == QCZ_MODE_FIXED ? cfg->level : 0;
    s->cache_on = (cfg->flags & QCZ_FLAG_CACHE) && cfg->mode != QCZ_MODE_PERBLOCK;
    s->cache_key_mask = (cfg->flags & QCZ_FLAG_CACHE_COLLIDE) ? 7ull : ~0ull;

    if (hip_stream) {
        s->stream = (hipStream_t)hip_stream;
    } else {
        hipError_t e = hipStreamCreate(&s->stream);
        if (e != hipSuccess) { delete s; return QCZ_E_DEVICE; }
        s->own_stream = true;
        (void)hipDeviceSynchronize();
    }
    int dev = 0, ncu = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    // one round of resident workgroups (three per CU for two-wavefront groups)
    s->grid_max = cfg->grid ? (int)cfg->grid : 3 * ncu;
    if (s->grid_max > kMaxGrid) s->grid_max = kMaxGrid;
    if (cfg->flags & QCZ_FLAG_AUTOTUNE) {
        for (int w : {2, 4, 8}) {
            if (s->C % (64 * w) != 0 || s->C / (64 * w) < 1) continue;
            for (int per_cu : {2, 3, 4, 6}) {
                const int g = std::min(per_cu * ncu, kMaxGrid);
                s->cands.push_back({w, g, 0.0, 0});
            }
        }
        s->tuning = !s->cands.empty();
    }

    s->block_levels.assign(s->nblocks, (uint8_t)(cfg->mode == QCZ_MODE_PERBLOCK ? cfg->level : 0));
    auto bail = [&](qcz_status st) {
        qcz_destroy(s);
        return st;
    };
    if (hipMemcpyAsync(s->blevel, s->block_levels.data(), s->nblocks, hipMemcpyHostToDevice, s->stream) != hipSuccess)
        return bail(QCZ_E_DEVICE);

    // |0...0>: chunk 0 holds amplitude 1 at index 0, every other chunk is zero
    // (Sec. 3.3: the state vectors are created in blocks and compressed).
    const size_t slot = (chunk_cap_bytes(s->C) + 3) & ~3u;
    double *raw = (double *)s->scratch;
    uint32_t *slots = (uint32_t *)(s->scratch + 2 * 8 * (size_t)s->C);
    uint32_t *sizes = (uint32_t *)(s->scratch + 2 * 8 * (size_t)s->C + 2 * slot);
    std::vector<double> init(2 * (size_t)s->C, 0.0);
    init[0] = 1.0;
    if (hipMemcpyAsync(raw, init.data(), init.size() * 8, hipMemcpyHostToDevice, s->stream) != hipSuccess)
        return bail(QCZ_E_DEVICE);
    if (qcz_encode_chunks(raw, (uint32_t)s->C, 2, 0, 0, slots, slot, sizes, s->stream) != QCZ_OK)
        return bail(QCZ_E_DEVICE);
    uint32_t hsz[2] = {0, 0};
    if (hipMemcpyAsync(hsz, sizes, 8, hipMemcpyDeviceToHost, s->stream) != hipSuccess) return bail(QCZ_E_DEVICE);
    if (hipStreamSynchronize(s->stream) != hipSuccess) return bail(QCZ_E_DEVICE);
    // streams start 16-byte aligned in the arena; the ledger counts 4-byte padded sizes
    const uint64_t p0 = alloc_bytes(hsz[0]), p1 = alloc_bytes(hsz[1]);
    if (hipMemcpyAsync(s->arena[0], slots, (hsz[0] + 3u) & ~3u, hipMemcpyDeviceToDevice, s->stream) != hipSuccess ||
        hipMemcpyAsync((uint8_t *)s->arena[0] + p0, (uint8_t *)slots + slot, (hsz[1] + 3u) & ~3u,
                       hipMemcpyDeviceToDevice, s->stream) != hipSuccess)
        return bail(QCZ_E_DEVICE);
    DevPtrs P = ptrs(s);
    if (launch_fill_table(P, (0ull << 16) | hsz[0], ((p0 / 4) << 16) | hsz[1], s->stream) != hipSuccess)
        return bail(QCZ_E_DEVICE);
    s->live = ((hsz[0] + 3u) & ~3ull) + ((hsz[1] + 3u) & ~3ull) * (s->nchunks - 1);
    s->min_c = s->max_c = s->live;
    if (reset_stripes(s, p0 + p1) != QCZ_OK) return bail(QCZ_E_DEVICE);
    if (hipStreamSynchronize(s->stream) != hipSuccess) return bail(QCZ_E_DEVICE);
    *out = s;
    return QCZ_OK;
}

void qcz_destroy(qcz_state *s)
{
    if (!s) return;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    clear_graphs(s);
    for (hipEvent_t ev : s->events) (void)hipEventDestroy(ev);
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

const char *qcz_last_error(const qcz_state *s) { return s ? s->err.c_str() : "null state"; }

uint64_t qcz_num_chunks(const qcz_state *s) { return s ? s->nchunks : 0; }
uint32_t qcz_chunk_doubles(const qcz_state *s) { return s ? (uint32_t)s->C : 0; }

qcz_status qcz_apply_gates(qcz_state *s, const qcz_gate *gates, size_t n_gates, size_t *applied)
{
    if (applied) *applied = 0;
    if (!s || (!gates && n_gates)) return QCZ_E_INVAL;
    if (s->broken) return fail(s, QCZ_E_STATE, "the state is invalid after a gate failed midway in ranges");
    for (size_t k = 0; k < n_gates; ++k)
        if (check_gate(s, gates[k]) != QCZ_OK)
            return fail(s, QCZ_E_INVAL, "malformed gate record " + std::to_string(k));
    size_t idx = 0;
    int compacted_for = -1;  // gate index a compaction was made for
    int swept_out = -1;      // gate index whose sweep ran out of arena
    int sweep_for = -1;      // gate index that did not fit after a compaction: sweep it
    std::vector<GateDesc> descs;
    while (idx < n_gates) {
        size_t B = std::min<size_t>((size_t)s->batch, n_gates - idx);
        if (s->sel_params) {
            // learned per-block levels: re-select every sel_period gates
            if (!s->sel_fresh || s->sel_since >= s->sel_period) {
                const size_t win = std::min<size_t>((size_t)s->sel_period, n_gates - idx);
                qcz_status st = select_levels(s, s->sel_params, s->sel_beta, mixing_mask(s, gates + idx, win), nullptr);
                if (st != QCZ_OK) return st;
                s->sel_fresh = true;
                s->sel_since = 0;
            }
            B = std::min<size_t>(B, (size_t)(s->sel_period - s->sel_since));
        }
        if (s->tuning) {
            const auto &c = s->cands[(size_t)s->tune_next];
            s->chunk_waves = c.waves;
            s->grid_max = c.grid;
        }
        descs.clear();
        for (size_t k = 0; k < B; ++k) descs.push_back(lower_gate(s, gates[idx + k], (int)k));
        B = through_first_run(s, descs);
        descs.resize(B);
        // A gate that does not fit beside the live streams sweeps into the
        // other arena when the state fits there (with the in-chunk gates
        // fused after it, under QCZ_FLAG_FUSE); a sweep the device stopped
        // for arena room falls back to compaction and job ranges below.
        if ((gates_that_fit(s, descs) == 0 || sweep_for == (int)idx) && sweepable(s, descs[0]) &&
            swept_out != (int)idx && sweep_may_fit(s)) {
            GateDesc launch;
            int kind = 0;
            size_t r = run_at(s, descs.data(), descs.size(), 0, launch, kind);
            if (kind == 0) {
                r = 1;
                launch = descs[0];
            }
            int reason = STOP_NONE;
            qcz_status st = apply_sweep(s, descs.data(), r, kind, launch, &reason);
            if (st != QCZ_OK) return st;
            if (reason == STOP_NONE) {
                idx += r;
                s->sel_since += r;
                if (applied) *applied = idx;
                continue;
            }
            if (reason == STOP_BUDGET) {
                if (s->level >= kLevels - 1)
                    return fail(s, QCZ_E_NOMEM, "compressed state exceeds the budget at the loosest level");
                s->level += 1;   // Sec. 3.7: relax the bound and redo the gate
                st = write_header(s);
                if (st != QCZ_OK) return st;
                continue;
            }
            if (reason != STOP_ARENA) return fail(s, QCZ_E_FORMAT, "a chunk table entry points outside the arena");
            swept_out = (int)idx;
            continue;
        }
        // Compact before a batch that is not expected to fit, so that a full
        // stripe seldom stops a batch midway (a stop costs a rollback and the
        // relaunch of the rest); if it still does not fit, launch the part
        // that does (at least one gate: the device-side check stays exact).
        if (gates_that_fit(s, descs) < B && s->bump > s->base) {
            qcz_status st = compact(s);
            if (st != QCZ_OK) return st;
        }
        const size_t fit = gates_that_fit(s, descs);
        if (fit == 0 && ranges_allowed(s) && descs[0].job_type != J_PERMUTE && descs[0].njobs > 1) {
            // one gate needs more arena room than is free: run it in job ranges
            qcz_status st = apply_in_ranges(s, descs[0]);
            if (st != QCZ_OK) return st;
            idx += 1;
            s->sel_since += 1;
            if (applied) *applied = idx;
            continue;
        }
        if (fit < B) {
            B = std::max<size_t>(1, fit);
            descs.resize(B);
        }
        const uint64_t live0 = s->live, bump0 = s->bump;
        qcz_status st = launch_batch(s, descs);
        if (st != QCZ_OK) return st;
        HIPCHK(s, hipMemcpyAsync(&s->hds, s->ds, offsetof(DevState, log) + B * sizeof(GateLog), hipMemcpyDeviceToHost,
                                 s->stream));
        HIPCHK(s, hipStreamSynchronize(s->stream));
        const DevState &h = s->hds;
        for (int k = 0; k < kStripes; ++k) s->stripe_fill[k] = h.stripe[k][0];
        if (!h.stop) {
            for (size_t k = 0; k < B; ++k) commit_logged(s, h, descs[k], (int)k);
            idx += B;
            s->sel_since += B;
            if (applied) *applied = idx;
            tune_step(s);
            continue;
        }
        const int sseq = h.stop_seq;
        const int reason = h.stop_reason;
        s->stats.stops += 1;
        for (int k = 0; k < sseq; ++k) commit_logged(s, h, descs[(size_t)k], k);
        s->sel_since += (uint64_t)sseq;
        // undo the stopped gate (a fused run's undo log covers every chunk)
        const bool run_stop = sseq < (int)s->run_first.size() && s->run_first[(size_t)sseq] == sseq &&
                              s->run_last[(size_t)sseq] > sseq;
        const GateDesc &gstop = descs[(size_t)sseq];
        const GateDesc dstop = run_stop ? s->run_desc[(size_t)sseq] : gstop;
        DevPtrs P = ptrs(s);
        const uint64_t work = dstop.job_type == J_PERMUTE ? dstop.njobs : launch_items(dstop);
        const int rg = (int)std::max<uint64_t>(1, std::min<uint64_t>((work + kWG - 1) / kWG, 65535));
        HIPCHK(s, launch_rollback(dstop, P, rg, s->stream));
        if (sseq == 0) { s->live = live0; s->bump = bump0; }
        idx += (size_t)sseq;
        if (applied) *applied = idx;
        if (reason == STOP_BUDGET) {
            if (s->level >= kLevels - 1) {
                (void)write_header(s);
                (void)hipStreamSynchronize(s->stream);
                return fail(s, QCZ_E_NOMEM, "compressed state exceeds the budget at the loosest level");
            }
            s->level += 1;   // Sec. 3.7: relax the bound and redo the gate
            st = write_header(s);
            if (st != QCZ_OK) return st;
        } else if (reason == STOP_ARENA) {
            st = write_header(s);
            if (st != QCZ_OK) return st;
            if (compacted_for == (int)idx) {
                // the gate's new streams do not fit beside the live ones even after
                // compaction: a sweep into the other arena, else job ranges
                if (swept_out != (int)idx && sweepable(s, gstop) && sweep_may_fit(s)) {
                    sweep_for = (int)idx;
                    continue;
                }
                if (!ranges_allowed(s) || gstop.job_type == J_PERMUTE || gstop.njobs < 2)
                    return fail(s, QCZ_E_NOMEM, "arena too small for one gate after compaction");
                st = apply_in_ranges(s, gstop);
                if (st != QCZ_OK) return st;
                idx += 1;
                s->sel_since += 1;
                if (applied) *applied = idx;
                continue;
            }
            st = compact(s);
            if (st != QCZ_OK) return st;
            compacted_for = (int)idx;
        } else {
            (void)write_header(s);
            (void)hipStreamSynchronize(s->stream);
            return fail(s, QCZ_E_FORMAT, "a chunk table entry points outside the arena");
        }
    }
    return QCZ_OK;
}

qcz_status qcz_footprint(qcz_state *s, qcz_footprint_t *out)
{
    if (!s || !out) return QCZ_E_INVAL;
    qcz_footprint_t f{};
    f.compressed_bytes = s->live;
    f.table_bytes = 8 * s->nchunks;
    f.total_bytes = f.compressed_bytes + f.table_bytes;
    f.raw_bytes = 1ull << (s->n + 4);
    f.arena_bytes = s->lay.arena_bytes;
    f.arena_used = s->bump;
    f.nchunks = s->nchunks;
    f.gates_applied = s->gates_applied;
    f.lossy_steps = s->lossy_steps;
    f.min_compressed = s->min_c;
    f.max_compressed = s->max_c;
    f.compactions = s->compactions;
    f.level = s->level;
    f.ratio = (double)f.raw_bytes / (double)f.total_bytes;
    f.fidelity_lower_bound = s->flb;
    *out = f;
    return QCZ_OK;
}

qcz_status qcz_export_state(qcz_state *s, void *host_buf, size_t cap, uint32_t *sizes, size_t *total)
{
    if (!s || !sizes || !total) return QCZ_E_INVAL;
    if (host_buf) {
        qcz_status st = compact(s);   // streams packed in chunk order from the arena's start
        if (st != QCZ_OK) return st;
    }
    std::vector<uint64_t> tab(s->nchunks);
    HIPCHK(s, hipMemcpyAsync(tab.data(), s->table, 8 * s->nchunks, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    uint64_t tot = 0;
    for (uint64_t c = 0; c < s->nchunks; ++c) {
        sizes[c] = (uint32_t)(tab[c] & 0xFFFFull);
        if (host_buf && (tab[c] >> 16) * 4 != tot) return fail(s, QCZ_E_STATE, "streams not packed after compaction");
        tot += alloc_bytes(sizes[c]);
    }
    *total = (size_t)tot;
    if (!host_buf) return QCZ_OK;
    if (cap < tot) return fail(s, QCZ_E_INVAL, "buffer smaller than the image");
    HIPCHK(s, hipMemcpyAsync(host_buf, s->arena[s->cur], tot, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    uint8_t *p = (uint8_t *)host_buf;
    uint64_t off = 0;
    for (uint64_t c = 0; c < s->nchunks; ++c) {   // compaction copies 4-byte words: clear the unit tails
        memset(p + off + sizes[c], 0, alloc_bytes(sizes[c]) - sizes[c]);
        off += alloc_bytes(sizes[c]);
    }
    return QCZ_OK;
}

qcz_status qcz_import_state(qcz_state *s, const void *host_buf, size_t len, const uint32_t *sizes)
{
    if (!s || !host_buf || !sizes) return QCZ_E_INVAL;
    const uint8_t *p = (const uint8_t *)host_buf;
    uint64_t off = 0, live = 0;
    std::vector<uint64_t> tab(s->nchunks);
    for (uint64_t c = 0; c < s->nchunks; ++c) {
        const uint32_t sz = sizes[c];
        if (sz < 4 || sz > chunk_cap_bytes(s->C) || off + alloc_bytes(sz) > len)
            return fail(s, QCZ_E_FORMAT, "stream size out of range");
        const uint32_t hdr = (uint32_t)p[off] | ((uint32_t)p[off + 1] << 8) | ((uint32_t)p[off + 2] << 16) |
                             ((uint32_t)p[off + 3] << 24);
        if (!header_ok(s, hdr, sz)) return fail(s, QCZ_E_FORMAT, "bad stream header");
        tab[c] = ((off / 4) << 16) | (uint64_t)sz;
        off += alloc_bytes(sz);
        live += (sz + 3u) & ~3u;
    }
    if (off != len) return fail(s, QCZ_E_FORMAT, "image length differs from the sizes");
    if (len > s->lay.arena_bytes) return fail(s, QCZ_E_NOMEM, "image larger than one arena");
    HIPCHK(s, hipMemcpyAsync(s->arena[s->cur], host_buf, len, hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipMemcpyAsync(s->table, tab.data(), 8 * s->nchunks, hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    s->live = live;
    s->min_c = s->max_c = live;
    // a fresh ledger at the configuration's level (qcz_resume restores a saved one); an
    // import also replaces a state left invalid by a failed ranged gate
    s->broken = false;
    s->level = s->cfg.mode == QCZ_MODE_FIXED ? s->cfg.level : 0;
    s->gates_applied = 0;
    s->lossy_steps = 0;
    s->flb = 1.0;
    clear_graphs(s);
    qcz_status st = reset_stripes(s, len);   // also writes the level to the device header
    if (st != QCZ_OK || s->cfg.mode != QCZ_MODE_PERBLOCK) return st;
    double mom[3];   // the per-block ledger divides by the stored state's squared norm
    st = qcz_moments(s, mom);
    if (st == QCZ_OK) s->norm2 = mom[2];
    return st;
}

qcz_status qcz_resume(qcz_state *s, const qcz_footprint_t *f)
{
    if (!s || !f) return QCZ_E_INVAL;
    if (f->raw_bytes != (1ull << (s->n + 4)) || f->nchunks != s->nchunks) return fail(s, QCZ_E_INVAL, "other shape");
    if (f->level < 0 || f->level >= kLevels || !(f->fidelity_lower_bound > 0.0 && f->fidelity_lower_bound <= 1.0) ||
        f->min_compressed > f->max_compressed || f->lossy_steps > f->gates_applied)
        return fail(s, QCZ_E_INVAL, "saved ledger out of range");
    if (s->cfg.mode == QCZ_MODE_PERBLOCK) return fail(s, QCZ_E_STATE, "per-block ledgers are not resumable");
    if (s->cfg.mode == QCZ_MODE_FIXED && f->level != s->cfg.level) return fail(s, QCZ_E_INVAL, "other fixed level");
    if (s->cfg.mode == QCZ_MODE_LOSSLESS && f->level != 0) return fail(s, QCZ_E_INVAL, "lossy level in lossless mode");
    if (f->compressed_bytes != s->live) return fail(s, QCZ_E_STATE, "imported streams differ from the saved size");
    s->level = f->level;
    s->gates_applied = f->gates_applied;
    s->lossy_steps = f->lossy_steps;
    s->min_c = f->min_compressed;
    s->max_c = f->max_compressed;
    s->flb = f->fidelity_lower_bound;
    clear_graphs(s);
    return write_header(s);   // the device copy of the level
}

qcz_status qcz_get_stats(qcz_state *s, qcz_stats_t *out)
{
    if (!s || !out) return QCZ_E_INVAL;
    *out = s->stats;
    out->chunk_waves = (uint32_t)s->chunk_waves;
    out->grid = (uint32_t)s->grid_max;
    out->tuning = s->tuning ? 1u : 0u;
    out->cache_on = s->cache_on ? 1u : 0u;
    return QCZ_OK;
}

qcz_status qcz_set_launch(qcz_state *s, uint32_t chunk_waves, uint32_t grid)
{
    if (!s) return QCZ_E_INVAL;
    if (chunk_waves) {
        if ((chunk_waves != 2 && chunk_waves != 4 && chunk_waves != 8) || s->C % (64 * (int)chunk_waves) != 0 ||
            (ent_state(s) && chunk_waves != 2))
            return fail(s, QCZ_E_INVAL, "unsupported chunk_waves");
        s->chunk_waves = (int)chunk_waves;
    }
    if (grid) {
        if (grid > (uint32_t)kMaxGrid) return fail(s, QCZ_E_INVAL, "grid too large");
        s->grid_max = (int)grid;
    }
    s->tuning = false;
    clear_graphs(s);
    return QCZ_OK;
}

qcz_status qcz_reset_stats(qcz_state *s)
{
    if (!s) return QCZ_E_INVAL;
    s->stats = qcz_stats_t{};
    return QCZ_OK;
}

qcz_status qcz_set_block_levels(qcz_state *s, const uint8_t *levels)
{
    if (!s || !levels) return QCZ_E_INVAL;
    if (s->cfg.mode != QCZ_MODE_PERBLOCK) return fail(s, QCZ_E_STATE, "block levels need QCZ_MODE_PERBLOCK");
    for (uint64_t b = 0; b < s->nblocks; ++b)
        if (levels[b] >= kLevels) return fail(s, QCZ_E_INVAL, "block level out of range");
    s->block_levels.assign(levels, levels + s->nblocks);
    HIPCHK(s, hipMemcpyAsync(s->blevel, s->block_levels.data(), s->nblocks, hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    clear_graphs(s);
    return QCZ_OK;
}

qcz_status qcz_decode_chunks_to(qcz_state *s, uint64_t first_chunk, uint64_t n_chunks, void *dev_out)
{
    if (!s || !dev_out || first_chunk > s->nchunks || n_chunks > s->nchunks - first_chunk) return QCZ_E_INVAL;
    if (n_chunks == 0) return QCZ_OK;
    GateDesc d{};
    single_kernel_chunks(s, d, n_chunks, first_chunk);
    IOPtrs io{};
    io.first = first_chunk;
    io.raw_out = (double *)dev_out;
    const int grid = (int)std::max<uint64_t>(1, std::min<uint64_t>(d.njobs, (uint64_t)s->grid_max));
    HIPCHK(s, launch_readout(d, ptrs(s), io, grid, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    return QCZ_OK;
}

qcz_status qcz_read_amplitudes(qcz_state *s, const uint64_t *idx, size_t k, double *out)
{
    if (!s || (k && (!idx || !out))) return QCZ_E_INVAL;
    const uint64_t N = 1ull << s->n;
    for (size_t i = 0; i < k; ++i)
        if (idx[i] >= N) return fail(s, QCZ_E_INVAL, "amplitude index out of range");
    std::vector<uint64_t> chunks;
    for (size_t i = 0; i < k; ++i) chunks.push_back(idx[i] >> s->cb);
    std::sort(chunks.begin(), chunks.end());
    chunks.erase(std::unique(chunks.begin(), chunks.end()), chunks.end());
    double *raw = (double *)s->scratch;
    uint64_t *list = (uint64_t *)(s->scratch + (size_t)kScratchChunks * 8 * (size_t)s->C);
    std::vector<double> host((size_t)kScratchChunks * (size_t)s->C);
    for (size_t base = 0; base < chunks.size(); base += kScratchChunks) {
        const size_t m = std::min<size_t>(kScratchChunks, chunks.size() - base);
        HIPCHK(s, hipMemcpyAsync(list, chunks.data() + base, m * 8, hipMemcpyHostToDevice, s->stream));
        GateDesc d{};
        single_kernel_chunks(s, d, m, 0);
        IOPtrs io{};
        io.list = list;
        io.raw_out = raw;
        const int grid = (int)std::max<uint64_t>(1, std::min<uint64_t>(d.njobs, (uint64_t)s->grid_max));
        HIPCHK(s, launch_readout(d, ptrs(s), io, grid, s->stream));
        HIPCHK(s, hipMemcpyAsync(host.data(), raw, m * 8 * (size_t)s->C, hipMemcpyDeviceToHost, s->stream));
        HIPCHK(s, hipStreamSynchronize(s->stream));
        for (size_t i = 0; i < k; ++i) {
            const uint64_t c = idx[i] >> s->cb;
            auto it = std::lower_bound(chunks.begin() + base, chunks.begin() + base + m, c);
            if (it == chunks.begin() + base + m || *it != c) continue;
            const size_t pos = (size_t)(it - (chunks.begin() + base));
            const uint64_t off = idx[i] & ((1ull << s->cb) - 1);
            out[2 * i] = host[pos * (size_t)s->C + 2 * off];
            out[2 * i + 1] = host[pos * (size_t)s->C + 2 * off + 1];
        }
    }
    return QCZ_OK;
}

qcz_status qcz_moments(qcz_state *s, double out[3])
{
    if (!s || !out) return QCZ_E_INVAL;
    GateDesc d{};
    single_kernel_chunks(s, d, s->nchunks, 0);
    IOPtrs io{};
    io.partials = s->partials;
    const int grid = (int)std::max<uint64_t>(1, std::min<uint64_t>(d.njobs, (uint64_t)kMomGrid));
    HIPCHK(s, launch_moments(d, ptrs(s), io, grid, s->stream));
    std::vector<double> h(4 * (size_t)grid);
    HIPCHK(s, hipMemcpyAsync(h.data(), s->partials, h.size() * 8, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    out[0] = out[1] = out[2] = 0.0;
    for (int g = 0; g < grid; ++g) {
        out[0] += h[4 * (size_t)g];
        out[1] += h[4 * (size_t)g + 1];
        out[2] += h[4 * (size_t)g + 2];
    }
    return QCZ_OK;
}

// SplitMix64 (Steele, Lea and Flood, 2014): output k of the generator whose
// state starts at `seed`.
static uint64_t splitmix64_at(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

qcz_status qcz_sample(qcz_state *s, uint64_t seed, size_t shots, uint64_t *out_idx)
{
    if (!s || (shots && !out_idx)) return QCZ_E_INVAL;
    if (shots == 0) return QCZ_OK;
    // squared norm of every chunk (device), prefix sums in chunk order (host)
    std::vector<double> cdf(s->nchunks);
    {
        double *cs = (double *)(s->pool + s->lay.cstats);
        const uint64_t per = std::min<uint64_t>(s->nchunks, kStatChunks);
        std::vector<double> rec((size_t)per * kChunkStats);
        for (uint64_t c0 = 0; c0 < s->nchunks; c0 += per) {
            const uint64_t m = std::min<uint64_t>(per, s->nchunks - c0);
            GateDesc d{};
            single_kernel_chunks(s, d, m, 0);
            d.block_shift = s->bl - s->cb;
            IOPtrs io{};
            io.first = c0;
            io.cstats = cs;
            const int grid = (int)std::max<uint64_t>(1, std::min<uint64_t>(d.njobs, (uint64_t)s->grid_max));
            HIPCHK(s, launch_chunk_stats(d, ptrs(s), io, grid, s->stream));
            HIPCHK(s, hipMemcpyAsync(rec.data(), cs, 8 * kChunkStats * m, hipMemcpyDeviceToHost, s->stream));
            HIPCHK(s, hipStreamSynchronize(s->stream));
            for (uint64_t k = 0; k < m; ++k) cdf[c0 + k] = rec[k * kChunkStats + CS_N2];
        }
    }
    double run = 0.0;
    uint64_t last_nz = 0;
    for (uint64_t c = 0; c < s->nchunks; ++c) {
        if (cdf[c] > 0.0) last_nz = c;
        run += cdf[c];
        cdf[c] = run;
    }
    const double total = run;
    if (!(total > 0.0)) return fail(s, QCZ_E_STATE, "the state has zero norm");
    // chunk of every shot
    std::vector<double> target(shots);
    std::vector<uint64_t> chunk_of(shots);
    for (size_t k = 0; k < shots; ++k) {
        const double u = (double)(splitmix64_at(seed, k) >> 11) * 0x1.0p-53;
        const double t = u * total;
        uint64_t c = (uint64_t)(std::upper_bound(cdf.begin(), cdf.end(), t) - cdf.begin());
        if (c >= s->nchunks) c = last_nz;
        chunk_of[k] = c;
        target[k] = t - (c ? cdf[c - 1] : 0.0);
    }
    std::vector<uint64_t> chunks(chunk_of);
    std::sort(chunks.begin(), chunks.end());
    chunks.erase(std::unique(chunks.begin(), chunks.end()), chunks.end());
    double *raw = (double *)s->scratch;
    uint64_t *list = (uint64_t *)(s->scratch + (size_t)kScratchChunks * 8 * (size_t)s->C);
    std::vector<double> host((size_t)kScratchChunks * (size_t)s->C);
    const uint64_t amps = (uint64_t)s->C / 2;
    for (size_t base = 0; base < chunks.size(); base += kScratchChunks) {
        const size_t m = std::min<size_t>(kScratchChunks, chunks.size() - base);
        HIPCHK(s, hipMemcpyAsync(list, chunks.data() + base, m * 8, hipMemcpyHostToDevice, s->stream));
        GateDesc d{};
        single_kernel_chunks(s, d, m, 0);
        IOPtrs io{};
        io.list = list;
        io.raw_out = raw;
        const int grid = (int)std::max<uint64_t>(1, std::min<uint64_t>(d.njobs, (uint64_t)s->grid_max));
        HIPCHK(s, launch_readout(d, ptrs(s), io, grid, s->stream));
        HIPCHK(s, hipMemcpyAsync(host.data(), raw, m * 8 * (size_t)s->C, hipMemcpyDeviceToHost, s->stream));
        HIPCHK(s, hipStreamSynchronize(s->stream));
        for (size_t k = 0; k < shots; ++k) {
            auto it = std::lower_bound(chunks.begin() + base, chunks.begin() + base + m, chunk_of[k]);
            if (it == chunks.begin() + base + m || *it != chunk_of[k]) continue;
            const double *a = host.data() + (size_t)(it - (chunks.begin() + base)) * (size_t)s->C;
            // first amplitude whose running |a|^2 passes the target (last nonzero one if rounding runs past)
            double acc = 0.0;
            uint64_t pick = amps, nz = 0;
            for (uint64_t i = 0; i < amps; ++i) {
                const double p = a[2 * i] * a[2 * i] + a[2 * i + 1] * a[2 * i + 1];
                if (p > 0.0) nz = i;
                acc += p;
                if (acc > target[k]) { pick = i; break; }
            }
            if (pick == amps) pick = nz;
            out_idx[k] = chunk_of[k] * amps + pick;
        }
    }
    return QCZ_OK;
}

qcz_status qcz_overlap(qcz_state *a, qcz_state *b, double *out_re, double *out_im)
{
    if (!a || !b || !out_re || !out_im) return QCZ_E_INVAL;
    if (a->n != b->n || a->C != b->C) return fail(a, QCZ_E_INVAL, "overlap needs the same qubits and chunk size");
    HIPCHK(a, hipStreamSynchronize(b->stream));
    double re = 0.0, im = 0.0;
    double *ra = (double *)a->scratch, *rb = (double *)b->scratch;
    std::vector<double> part(512);
    for (uint64_t c0 = 0; c0 < a->nchunks; c0 += kScratchChunks) {
        const uint64_t m = std::min<uint64_t>(kScratchChunks, a->nchunks - c0);
        GateDesc d{};
        single_kernel_chunks(a, d, m, 0);
        d.entropy = ent_state(a) | ent_state(b);   // entropy kernels decode both kinds of stream
        IOPtrs io{};
        io.first = c0;
        io.raw_out = ra;
        const int grid = (int)std::max<uint64_t>(1, std::min<uint64_t>(d.njobs, (uint64_t)a->grid_max));
        HIPCHK(a, launch_readout(d, ptrs(a), io, grid, a->stream));
        io.raw_out = rb;
        HIPCHK(a, launch_readout(d, ptrs(b), io, grid, a->stream));
        const uint64_t npairs = m * (uint64_t)a->C / 2;
        const int dg = (int)std::min<uint64_t>(256, (npairs + kWG - 1) / kWG);
        HIPCHK(a, launch_dot(ra, rb, npairs, a->partials, dg, a->stream));
        HIPCHK(a, hipMemcpyAsync(part.data(), a->partials, 16 * (size_t)dg, hipMemcpyDeviceToHost, a->stream));
        HIPCHK(a, hipStreamSynchronize(a->stream));
        for (int g = 0; g < dg; ++g) { re += part[2 * (size_t)g]; im += part[2 * (size_t)g + 1]; }
    }
    *out_re = re;
    *out_im = im;
    return QCZ_OK;
}

qcz_status qcz_export_chunk(qcz_state *s, uint64_t chunk, void *host_buf, size_t cap, size_t *len)
{
    if (!s || !host_buf || !len || chunk >= s->nchunks) return QCZ_E_INVAL;
    uint64_t e = 0;
    HIPCHK(s, hipMemcpyAsync(&e, s->table + chunk, 8, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    const size_t size = (size_t)(e & 0xFFFF);
    const uint64_t off = e >> 16;
    *len = size;
    if (size > cap) return fail(s, QCZ_E_INVAL, "export buffer too small");
    if (off * 4 + size > s->lay.arena_bytes) return fail(s, QCZ_E_FORMAT, "chunk entry outside the arena");
    HIPCHK(s, hipMemcpyAsync(host_buf, (uint8_t *)s->arena[s->cur] + off * 4, size, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    return QCZ_OK;
}

qcz_status qcz_import_chunk(qcz_state *s, uint64_t chunk, const void *host_buf, size_t len)
{
    if (!s || !host_buf || chunk >= s->nchunks) return QCZ_E_INVAL;
    if (len < 4 || len > chunk_cap_bytes(s->C)) return fail(s, QCZ_E_FORMAT, "stream length out of range");
    const uint8_t *p = (const uint8_t *)host_buf;
    const uint32_t hdr = (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
    if (!header_ok(s, hdr, len)) return fail(s, QCZ_E_FORMAT, "bad stream header");
    const uint64_t pad = (len + 3) & ~(size_t)3;   // ledger size
    const uint64_t room_needed = alloc_bytes((uint32_t)len);   // arena allocation (16-byte units)
    auto emptiest = [&]() {
        int best = 0;
        for (int k = 1; k < s->nstripes; ++k)
            if (s->stripe_fill[k] < s->stripe_fill[best]) best = k;
        return best;
    };
    int sk = emptiest();
    if (s->stripe_fill[sk] + room_needed > s->stripe_size) {
        qcz_status st = compact(s);
        if (st != QCZ_OK) return st;
        sk = emptiest();
        if (s->stripe_fill[sk] + room_needed > s->stripe_size) return fail(s, QCZ_E_NOMEM, "arena full");
    }
    const uint64_t where = s->base + (uint64_t)sk * s->stripe_size + s->stripe_fill[sk];
    uint64_t old = 0;
    HIPCHK(s, hipMemcpyAsync(&old, s->table + chunk, 8, hipMemcpyDeviceToHost, s->stream));
    std::vector<uint8_t> tmp(pad, 0);
    memcpy(tmp.data(), host_buf, len);
    HIPCHK(s, hipMemcpyAsync((uint8_t *)s->arena[s->cur] + where, tmp.data(), pad, hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    const uint64_t entry = ((where / 4) << 16) | (uint64_t)len;
    HIPCHK(s, hipMemcpyAsync(s->table + chunk, &entry, 8, hipMemcpyHostToDevice, s->stream));
    const uint64_t old_pad = ((old & 0xFFFF) + 3) & ~3ull;
    s->live = s->live + pad - old_pad;
    s->stripe_fill[sk] += room_needed;
    s->bump += room_needed;
    s->hds.stripe[sk][0] = s->stripe_fill[sk];
    HIPCHK(s, hipMemcpyAsync(&s->ds->stripe[sk][0], &s->hds.stripe[sk][0], 8, hipMemcpyHostToDevice, s->stream));
    qcz_status st = write_header(s);
    if (st != QCZ_OK) return st;
    HIPCHK(s, hipStreamSynchronize(s->stream));
    clear_graphs(s);
    return QCZ_OK;
}

qcz_status qcz_chunk_sizes(qcz_state *s, uint32_t *out_sizes)
{
    if (!s || !out_sizes) return QCZ_E_INVAL;
    std::vector<uint64_t> t(s->nchunks);
    HIPCHK(s, hipMemcpyAsync(t.data(), s->table, 8 * s->nchunks, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    for (uint64_t c = 0; c < s->nchunks; ++c) out_sizes[c] = (uint32_t)(t[c] & 0xFFFF);
    return QCZ_OK;
}

qcz_status qcz_encode_chunks(const void *dev_in, uint32_t C, uint64_t n_chunks, int level, uint32_t codec_flags,
                             void *dev_slots, size_t slot_bytes, uint32_t *dev_sizes, void *hip_stream)
{
    if (!dev_in || !dev_slots || !dev_sizes) return QCZ_E_INVAL;
    if (C < (uint32_t)kCMin || C > (uint32_t)kCMax || (C & (C - 1)) || level < 0 || level >= kLevels) return QCZ_E_INVAL;
    if (codec_flags == QCZ_CODEC_PREDICT) {
        if (C < 256 || level < 1 || slot_bytes < pred_cap_bytes((int)C) || (slot_bytes & 3)) return QCZ_E_INVAL;
        if (n_chunks == 0) return QCZ_OK;
        return launch_pred_encode((const double *)dev_in, (int)C, level, n_chunks, (uint32_t *)dev_slots, slot_bytes / 4,
                                  dev_sizes, (hipStream_t)hip_stream) == hipSuccess
                   ? QCZ_OK
                   : QCZ_E_DEVICE;
    }
    if ((codec_flags & ~(QCZ_CODEC_ENTROPY | QCZ_CODEC_RESHUFFLE)) ||
        ((codec_flags & QCZ_CODEC_ENTROPY) && C != (uint32_t)kCMax))
        return QCZ_E_INVAL;
    if (slot_bytes < chunk_cap_bytes((int)C) || (slot_bytes & 3)) return QCZ_E_INVAL;
    if (n_chunks == 0) return QCZ_OK;
    GateDesc d{};
    d.job_type = J_SINGLE;
    d.nitems = n_chunks;
    d.njobs = (n_chunks + 1) / 2;
    int bits = 0;
    while ((1ull << bits) < n_chunks) ++bits;
    d.nchunk_bits = bits;
    d.fixed_level = level;
    d.entropy = (codec_flags & QCZ_CODEC_ENTROPY) ? 1 : 0;
    d.reshuffle = (codec_flags & QCZ_CODEC_RESHUFFLE) ? 1 : 0;
    DevPtrs P{};
    P.C = (int)C;
    int cb = 0;
    while ((2u << cb) < C) ++cb;
    P.cb = cb;
    IOPtrs io{};
    io.raw_in = (const double *)dev_in;
    io.slots_out = (uint32_t *)dev_slots;
    io.sizes_out = dev_sizes;
    io.slot_words = slot_bytes / 4;
    const int grid = (int)std::min<uint64_t>(d.njobs, 4096);
    if (launch_encode_raw(d, P, io, grid, (hipStream_t)hip_stream) != hipSuccess) return QCZ_E_DEVICE;
    return QCZ_OK;
}

qcz_status qcz_decode_chunks(const void *dev_slots, size_t slot_bytes, const uint32_t *dev_sizes, uint32_t C,
                             uint64_t n_chunks, void *dev_out, void *hip_stream)
{
    if (!dev_slots || !dev_sizes || !dev_out) return QCZ_E_INVAL;
    if (C < (uint32_t)kCMin || C > (uint32_t)kCMax || (C & (C - 1)) || (slot_bytes & 3) || slot_bytes < 4)
        return QCZ_E_INVAL;
    if (n_chunks == 0) return QCZ_OK;
    GateDesc d{};
    d.job_type = J_SINGLE;
    d.nitems = n_chunks;
    d.njobs = (n_chunks + 1) / 2;
    int bits = 0;
    while ((1ull << bits) < n_chunks) ++bits;
    d.nchunk_bits = bits;
    d.fixed_level = 0;
    d.entropy = C == (uint32_t)kCMax ? 1 : 0;   // those kernels decode streams with and without the entropy stage
    DevPtrs P{};
    P.C = (int)C;
    IOPtrs io{};
    io.slots_in = (const uint32_t *)dev_slots;
    io.sizes_in = dev_sizes;
    io.slot_words = slot_bytes / 4;
    io.raw_out = (double *)dev_out;
    const int grid = (int)std::min<uint64_t>(d.njobs, 4096);
    if (launch_decode_slots(d, P, io, grid, (hipStream_t)hip_stream) != hipSuccess) return QCZ_E_DEVICE;
    if (C >= 256 && launch_pred_decode((const uint32_t *)dev_slots, slot_bytes / 4, dev_sizes, (int)C, n_chunks,
                                       (double *)dev_out, (hipStream_t)hip_stream) != hipSuccess)
        return QCZ_E_DEVICE;
    return QCZ_OK;
}

size_t qcz_chunk_cap_codec(uint32_t C, uint32_t codec_flags)
{
    if (C < (uint32_t)kCMin || C > (uint32_t)kCMax || (C & (C - 1))) return 0;
    if (codec_flags == QCZ_CODEC_PREDICT) return C >= 256 ? pred_cap_bytes((int)C) : 0;
    if (codec_flags & ~(QCZ_CODEC_ENTROPY | QCZ_CODEC_RESHUFFLE)) return 0;
    return chunk_cap_bytes((int)C);
}

// ---------------------------------------------------------------------------
// per-block level selection
// ---------------------------------------------------------------------------
qcz_status qcz_block_stats(qcz_state *s, double beta, uint64_t mix_mask, float *dev_features, double *dev_norms)
{
    if (!s || !dev_features || !(beta >= 0.0) || (mix_mask >> (s->n - s->bl))) return QCZ_E_INVAL;
    qcz_status st = block_stats(s, beta, mix_mask, dev_features, dev_norms);
    if (st != QCZ_OK) return st;
    HIPCHK(s, hipStreamSynchronize(s->stream));
    return QCZ_OK;
}

qcz_status qcz_block_level_sizes(qcz_state *s, uint64_t *dev_sizes)
{
    if (!s || !dev_sizes) return QCZ_E_INVAL;
    HIPCHK(s, launch_zero_u64(dev_sizes, (uint64_t)kLevels * s->nblocks, s->stream));
    GateDesc d{};
    single_kernel_chunks(s, d, s->nchunks, 0);
    d.block_shift = s->bl - s->cb;
    IOPtrs io{};
    io.lsizes = dev_sizes;
    const int grid = (int)std::max<uint64_t>(1, std::min<uint64_t>(d.njobs, (uint64_t)s->grid_max));
    HIPCHK(s, launch_level_sizes(d, ptrs(s), io, grid, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    return QCZ_OK;
}

qcz_status qcz_label_levels(const uint64_t *sizes, const double *w, uint64_t nblocks, double beta, uint64_t mix_mask,
                            uint8_t *levels)
{
    if ((nblocks && (!sizes || !w || !levels)) || !(beta >= 0.0) || (mix_mask & ~(nblocks - 1)) ||
        (nblocks & (nblocks - 1)))
        return QCZ_E_INVAL;
    for (uint64_t b = 0; b < nblocks; ++b)
        if (!(w[b] >= 0.0)) return QCZ_E_INVAL;
    if (nblocks == 0) return QCZ_OK;
    const double lim = beta * (1.0 + std::ldexp(1.0, -20));
    const Cosets cs = make_cosets(w, nblocks, mix_mask);
    const size_t nc = cs.ids.size();
    // smallest level <= cap of each block (lowest on ties) and the coset's bytes under each cap
    auto capped = [&](uint64_t b, int cap) {
        int best = 0;
        for (int l = 1; l <= cap; ++l)
            if (sizes[b * kLevels + l] < sizes[b * kLevels + best]) best = l;
        return best;
    };
    std::vector<double> cost(nc * kLevels, 0.0);
    for (size_t k = 0; k < nc; ++k)
        for (int cap = 0; cap < kLevels; ++cap) {
            double t = 0.0;
            for (uint64_t i = cs.start[k]; i < cs.start[k + 1]; ++i) {
                const uint64_t b = cs.mem[i];
                t += (double)sizes[b * kLevels + capped(b, cap)];
            }
            cost[k * kLevels + cap] = t;
        }
    std::vector<int> caps(nc, 0);
    auto choose = [&](double lam) {
        double t = 0.0;
        for (size_t k = 0; k < nc; ++k) {
            int best = 0;
            double bc = 0.0;
            for (int cap = 0; cap < kLevels; ++cap) {
                const double v = cost[k * kLevels + cap] + lam * (cs.W[k] * kDelta[cap]);
                if (cap == 0 || v < bc) { best = cap; bc = v; }
            }
            caps[k] = best;
        }
        for (size_t k = 0; k < nc; ++k) t += cs.W[k] * kDelta[caps[k]];
        return t <= lim;
    };
    // candidate multipliers: 0 and every value where a coset's choice can change
    std::vector<double> lam{0.0};
    for (size_t k = 0; k < nc; ++k) {
        if (cs.W[k] <= 0.0) continue;
        for (int lo = 0; lo < kLevels; ++lo)
            for (int hi = lo + 1; hi < kLevels; ++hi) {
                const double d = cost[k * kLevels + lo] - cost[k * kLevels + hi];
                if (d > 0.0) lam.push_back(d / (cs.W[k] * (kDelta[hi] - kDelta[lo])));
            }
    }
    std::sort(lam.begin(), lam.end());
    lam.erase(std::unique(lam.begin(), lam.end()), lam.end());
    // the budget use falls as the multiplier grows: smallest feasible candidate by bisection
    size_t lo = 0, hi = lam.size();
    while (lo < hi) {
        const size_t mid = lo + (hi - lo) / 2;
        if (choose(lam[mid])) hi = mid;
        else lo = mid + 1;
    }
    if (lo == lam.size()) {
        for (uint64_t b = 0; b < nblocks; ++b) levels[b] = 0;
        return QCZ_OK;
    }
    choose(lam[lo]);
    for (size_t k = 0; k < nc; ++k)
        for (uint64_t i = cs.start[k]; i < cs.start[k + 1]; ++i) levels[cs.mem[i]] = (uint8_t)capped(cs.mem[i], caps[k]);
    return QCZ_OK;
}

qcz_status qcz_project_levels(const double *w, uint64_t nblocks, double beta, uint64_t mix_mask, uint8_t *levels)
{
    if ((nblocks && (!w || !levels)) || !(beta >= 0.0) || (mix_mask & ~(nblocks - 1)) || (nblocks & (nblocks - 1)))
        return QCZ_E_INVAL;
    for (uint64_t b = 0; b < nblocks; ++b)
        if (!(w[b] >= 0.0) || levels[b] >= kLevels) return QCZ_E_INVAL;
    if (nblocks == 0) return QCZ_OK;
    project(w, nblocks, beta, mix_mask, levels);
    return QCZ_OK;
}

size_t qcz_mlp_workspace_bytes(uint64_t n_samples) { return n_samples ? mlp_workspace_bytes(n_samples) : 0; }

qcz_status qcz_mlp_forward(const float *dev_params, const float *dev_x, uint64_t n_samples, float *dev_probs,
                           uint8_t *dev_levels, void *hip_stream)
{
    if (!dev_params || (n_samples && !dev_x)) return QCZ_E_INVAL;
    if (launch_mlp_forward(dev_params, dev_x, n_samples, dev_probs, dev_levels, (hipStream_t)hip_stream) !=
        hipSuccess)
        return QCZ_E_DEVICE;
    return QCZ_OK;
}

qcz_status qcz_mlp_train_step(float *dev_params, float *dev_m, float *dev_v, const float *dev_x,
                              const uint8_t *dev_labels, uint64_t n_samples, float lr, uint32_t step,
                              float *dev_grad, float *dev_loss, void *dev_work, size_t work_bytes, void *hip_stream)
{
    if (!dev_params || !dev_x || !dev_labels || !dev_work || n_samples == 0) return QCZ_E_INVAL;
    if (step > 0 && (!dev_m || !dev_v)) return QCZ_E_INVAL;
    if (work_bytes < mlp_workspace_bytes(n_samples)) return QCZ_E_INVAL;
    if (launch_mlp_train(dev_params, dev_m, dev_v, dev_x, dev_labels, n_samples, lr, step, dev_grad, dev_loss,
                         dev_work, (hipStream_t)hip_stream) != hipSuccess)
        return QCZ_E_DEVICE;
    return QCZ_OK;
}

qcz_status qcz_mlp_train_step_noalloc(float *dev_params, float *dev_m, float *dev_v, const float *dev_x,
                                      const uint8_t *dev_labels, uint64_t n_samples, float lr, uint32_t step,
                                      float *dev_grad, float *dev_loss, void *hip_stream)
{
    if (!dev_params || !dev_x || !dev_labels || n_samples == 0) return QCZ_E_INVAL;
    if (step > 0 && (!dev_m || !dev_v)) return QCZ_E_INVAL;
    if (n_samples > (uint64_t)QCZ_MLP_NOALLOC_MAX_SAMPLES) return QCZ_E_NOMEM;
    static_assert(QCZ_MLP_NOALLOC_MAX_SAMPLES == kMlpStaticSamples, "header and kernels agree on the limit");
    void *ws = nullptr;
    size_t bytes = 0;
    if (mlp_static_workspace(&ws, &bytes) != hipSuccess || bytes < mlp_workspace_bytes(n_samples))
        return QCZ_E_DEVICE;
    if (launch_mlp_train(dev_params, dev_m, dev_v, dev_x, dev_labels, n_samples, lr, step, dev_grad, dev_loss, ws,
                         (hipStream_t)hip_stream) != hipSuccess)
        return QCZ_E_DEVICE;
    return QCZ_OK;
}

qcz_status qcz_select_levels(qcz_state *s, const float *dev_params, double beta, uint64_t mix_mask,
                             uint8_t *out_levels)
{
    if (!s || !dev_params || !(beta >= 0.0) || (mix_mask >> (s->n - s->bl))) return QCZ_E_INVAL;
    qcz_status st = select_levels(s, dev_params, beta, mix_mask, out_levels);
    if (st == QCZ_OK) clear_graphs(s);
    return st;
}

qcz_status qcz_set_selector(qcz_state *s, const float *dev_params, double beta, uint32_t period)
{
    if (!s || (dev_params && (!(beta >= 0.0) || period == 0))) return QCZ_E_INVAL;
    if (dev_params && s->cfg.mode != QCZ_MODE_PERBLOCK)
        return fail(s, QCZ_E_STATE, "level selection needs QCZ_MODE_PERBLOCK");
    s->sel_params = dev_params;
    s->sel_beta = beta;
    s->sel_period = period;
    s->sel_since = 0;
    s->sel_fresh = false;
    return QCZ_OK;
}

qcz_status qcz_copy_state(qcz_state *dst, qcz_state *src)
{
    if (!dst || !src || dst == src || dst->n != src->n || dst->bl != src->bl || dst->cfg.mode != src->cfg.mode)
        return QCZ_E_INVAL;
    // compact the source first: its live streams then fill [0, base) of its arena
    // (streams appended since the last compaction sit in stripes spread over the arena)
    if (src->bump > src->base) {
        qcz_status st = compact(src);
        if (st != QCZ_OK) return fail(dst, st, "compacting the source: " + src->err);
    }
    const uint64_t used = src->base;
    if (used > dst->lay.arena_bytes) return fail(dst, QCZ_E_NOMEM, "destination arena smaller than the source's streams");
    HIPCHK(dst, hipStreamSynchronize(src->stream));
    HIPCHK(dst, hipMemcpyAsync(dst->table, src->table, 8 * src->nchunks, hipMemcpyDeviceToDevice, dst->stream));
    if (used)
        HIPCHK(dst, hipMemcpyAsync(dst->arena[dst->cur], src->arena[src->cur], used, hipMemcpyDeviceToDevice,
                                   dst->stream));
    dst->level = src->level;
    dst->live = src->live;
    dst->block_levels = src->block_levels;
    dst->flb = src->flb;
    dst->norm2 = src->norm2;
    dst->gates_applied = src->gates_applied;
    dst->lossy_steps = src->lossy_steps;
    dst->min_c = src->min_c;
    dst->max_c = src->max_c;
    HIPCHK(dst, hipMemcpyAsync(dst->blevel, dst->block_levels.data(), dst->nblocks, hipMemcpyHostToDevice,
                               dst->stream));
    qcz_status st = reset_stripes(dst, used);
    if (st != QCZ_OK) return st;
    HIPCHK(dst, hipStreamSynchronize(dst->stream));
    return QCZ_OK;
}

uint64_t qcz_mixing_mask(const qcz_state *s, const qcz_gate *gates, size_t n_gates)
{
    if (!s || (n_gates && !gates)) return 0;
    return mixing_mask(s, gates, n_gates);
}

}  // extern "C"

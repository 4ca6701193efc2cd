// HIP kernels (gfx950) of the compressed state-vector simulator.
//
// The state is a table of independently compressed chunks of C interleaved
// doubles (re a_k, im a_k, ...).  One gate is one kernel: every workgroup
// takes jobs of two chunk positions (a pair whose amplitudes differ in the
// target bit, or two independent chunks), and per job
//   1. stages the compressed chunks from HBM into LDS (coalesced words),
//   2. decodes them (Solution C of Sec. 4.2: two-bit leading-byte codes and
//      truncated residuals, rebuilt with wavefront scans),
//   3. applies the 2x2 unitary of Eq. (6) / (7) in fp64,
//   4. re-encodes each chunk at the gate's error level (Eq. (12) truncation,
//      XOR leading-byte codes, CONST2 / PACK / SPARSE lossless stage) into
//      LDS, and
//   5. appends the new stream to the arena with one atomic and updates the
//      chunk table, keeping the previous entry in an undo log.
// Decompressed data never leaves LDS, so the per-gate HBM traffic is the
// compressed bytes read plus the compressed bytes written.
//
// Every routine that carries a barrier is executed by all 256 threads of a
// workgroup in the same order; per-slot differences are data, not control
// flow around barriers.
#include "qcz_internal.h"

#include <hip/hip_ext.h>

namespace qcz {

// Sig_Bit_Count of Eq. (12) for binary64 (12 sign/exponent bits minus the
// exponent of the bound) per level: lossless, 1e-5, 1e-4, 1e-3, 1e-2, 1e-1.
// Selected in registers: the level is a per-lane value, and a table in
// memory would cost a load and a wait for every outstanding memory access.
__device__ __forceinline__ int sig_bits(int lev)
{
    return lev == 1 ? 29 : lev == 2 ? 26 : lev == 3 ? 22 : lev == 4 ? 19 : lev == 5 ? 16 : 64;
}

enum { SRC_ARENA = 0, SRC_RAW = 1, SRC_SLOTS = 2 };
enum { DST_ARENA = 0, DST_RAW = 1, DST_SLOTS = 2, DST_MOMENTS = 3, DST_CSTATS = 4, DST_LSIZES = 5 };

// delta of each level (0 for lossless): the per-value relative bound of Sec. 3.7
__device__ __forceinline__ double level_delta(int lev)
{
    return lev == 1 ? 1e-5 : lev == 2 ? 1e-4 : lev == 3 ? 1e-3 : lev == 4 ? 1e-2 : lev == 5 ? 1e-1 : 0.0;
}

// ---------------------------------------------------------------------------
// bit helpers.  A value is handled as its two 32-bit words (hi, lo).  At every
// lossy level Sig_Bit_Count <= 29, so a truncated value lives entirely in its
// high word; the leading-byte code looks at the top three bytes only, which
// are high-word bits as well.  Only lossless chunks carry low words.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t d2u(double x) { return (uint64_t)__double_as_longlong(x); }
__device__ __forceinline__ double u2d(uint64_t b) { return __longlong_as_double((long long)b); }

__device__ __forceinline__ uint32_t lead_bytes(uint32_t cur_hi, uint32_t prev_hi)
{
    // (| 1: the count never sees zero, so no zero fix-up; equal words give 3)
    const uint32_t L = (uint32_t)__clz((int)((cur_hi ^ prev_hi) | 1u)) >> 3;
    return L < 3u ? L : 3u;
}

__device__ __forceinline__ uint32_t resid_bits(int K, uint32_t L)
{
    const int r = K - 8 * (int)L;
    return r > 0 ? (uint32_t)r : 0u;
}

// residual bits of n values whose two-bit codes are packed in `codes`
// (positions past n hold code 0 and are not counted)
__device__ __forceinline__ uint32_t resid_total(uint32_t codes, int K, uint32_t n)
{
    const uint32_t lo = codes & 0x55555555u, hi = (codes >> 1) & 0x55555555u;
    const uint32_t n3 = __popc(lo & hi), n2 = __popc(hi & ~lo), n1 = __popc(lo & ~hi);
    return (n - n1 - n2 - n3) * resid_bits(K, 0) + n1 * resid_bits(K, 1) + n2 * resid_bits(K, 2) +
           n3 * resid_bits(K, 3);
}

__device__ __forceinline__ uint32_t low_mask32(uint32_t r) { return r >= 32u ? ~0u : ((1u << r) - 1u); }
__device__ __forceinline__ uint32_t sig_mask_hi(int K) { return K >= 32 ? ~0u : ~((1u << (32 - K)) - 1u); }

__device__ __forceinline__ bool subnormal(uint32_t h, uint32_t l)
{
    return ((h >> 20) & 0x7FFu) == 0 && ((h & 0xFFFFFu) | l) != 0;
}

// the same test on a double (one class comparison: positive or negative subnormal)
__device__ __forceinline__ bool is_subnormal(double x) { return __builtin_isfpclass(x, 0x0090); }

__device__ __forceinline__ int clampw(int i) { return i < kBufWords - 1 ? i : kBufWords - 1; }
// first of N consecutive words read together (one ds_read2 for N = 2)
template <int N>
__device__ __forceinline__ int clampn(int i) { return i < kBufWords - N ? i : kBufWords - N; }
static_assert(kBufWords % 4 == 0, "stream buffers are cleared in 16-byte units");

// LDS position of value i of a decoded chunk: one pad double after every 16
// values, so that threads owning 16 consecutive values each start in
// different banks (unpadded, a wavefront's accesses to its values all fall
// into the same bank)
__device__ __forceinline__ int vpos(int i) { return i + (i >> 4); }

// bits [sh, sh+32) of the 64-bit word pair (hi:lo)
__device__ __forceinline__ uint32_t fshr(uint32_t hi, uint32_t lo, uint32_t sh)
{
    return __builtin_amdgcn_alignbit(hi, lo, sh);
}

// Copy `words` words of a 16-byte aligned stream (its arena allocation is a
// whole number of 16-byte units) into 16-byte aligned LDS, four 16-byte
// loads in flight per thread; the last unit may carry up to three words past
// the stream, which belong to its allocation.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <int G>
__device__ __forceinline__ void stage_units(uint32_t *dst, const uint32_t *src, uint32_t words, int lt)
{
    const uint32_t units = (words + 3u) >> 2;
    const u32x4 *s4 = reinterpret_cast<const u32x4 *>(src);
    u32x4 *d4 = reinterpret_cast<u32x4 *>(dst);
    for (uint32_t base = (uint32_t)lt; base < units; base += 4u * G) {
        u32x4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t w = base + (uint32_t)u * G;
            v[u] = (w < units) ? __builtin_nontemporal_load(s4 + w) : u32x4{0u, 0u, 0u, 0u};
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t w = base + (uint32_t)u * G;
            if (w < units) d4[w] = v[u];
        }
    }
}

// Two streams at once (each as in stage_units, `on` selecting which are
// copied): the loads of both are in flight together, one HBM round trip for
// streams of up to 4 G units.
template <int G>
__device__ __forceinline__ void stage_units2(uint32_t *dst0, const uint32_t *src0, uint32_t words0, bool on0,
                                             uint32_t *dst1, const uint32_t *src1, uint32_t words1, bool on1, int lt)
{
    const uint32_t units0 = on0 ? (words0 + 3u) >> 2 : 0u, units1 = on1 ? (words1 + 3u) >> 2 : 0u;
    const uint32_t units = units0 > units1 ? units0 : units1;
    const u32x4 *a4 = reinterpret_cast<const u32x4 *>(src0);
    const u32x4 *b4 = reinterpret_cast<const u32x4 *>(src1);
    u32x4 *c4 = reinterpret_cast<u32x4 *>(dst0);
    u32x4 *d4 = reinterpret_cast<u32x4 *>(dst1);
    for (uint32_t base = (uint32_t)lt; base < units; base += 4u * G) {
        u32x4 v[4], y[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t w = base + (uint32_t)u * G;
            v[u] = (w < units0) ? __builtin_nontemporal_load(a4 + w) : u32x4{0u, 0u, 0u, 0u};
            y[u] = (w < units1) ? __builtin_nontemporal_load(b4 + w) : u32x4{0u, 0u, 0u, 0u};
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t w = base + (uint32_t)u * G;
            if (w < units0) c4[w] = v[u];
            if (w < units1) d4[w] = y[u];
        }
    }
}

// Workgroup barrier that orders LDS only: pending global stores and loads
// are not waited for (no thread of the workgroup reads them back).
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Copy `words` words from global memory into LDS with eight loads in flight
// per thread (one HBM round trip per 1024 words).
template <int G>
__device__ __forceinline__ void stage_words(uint32_t *dst, const uint32_t *src, uint32_t words, int lt)
{
    for (uint32_t base = (uint32_t)lt; base < words; base += 8u * G) {
        uint32_t v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint32_t w = base + (uint32_t)u * G;
            v[u] = (w < words) ? __builtin_nontemporal_load(src + w) : 0u;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint32_t w = base + (uint32_t)u * G;
            if (w < words) dst[w] = v[u];
        }
    }
}

// ---------------------------------------------------------------------------
// scans.  A group is the 128 threads (two wavefronts) of one chunk slot.
// Wavefront scans use DPP row shifts (1, 2, 4, 8) and row broadcasts (15,
// 31); the two wavefronts of a group meet through LDS with one barrier.
// Each call site owns its LDS slot, so no second barrier is needed before the
// slot is reused (the next use is a job later, many barriers away).
// ---------------------------------------------------------------------------
template <int CTRL, int RMASK>
__device__ __forceinline__ uint32_t dpp0(uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, RMASK, 0xF, false);
}

__device__ __forceinline__ uint32_t wave_incl_add(uint32_t x)
{
    x += dpp0<0x111, 0xF>(x);
    x += dpp0<0x112, 0xF>(x);
    x += dpp0<0x114, 0xF>(x);
    x += dpp0<0x118, 0xF>(x);
    x += dpp0<0x142, 0xA>(x);
    x += dpp0<0x143, 0xC>(x);
    return x;
}

// exclusive sum over the group (WPG wavefronts), and the group total
template <int WPG>
__device__ __forceinline__ void gscan_add(uint32_t v, uint32_t *slot, uint32_t &ex, uint32_t &tot)
{
    const uint32_t x = wave_incl_add(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 63) slot[w] = x;
    lds_barrier();
    const int g0 = w - (w % WPG);
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < WPG; ++i) {
        const uint32_t t = slot[g0 + i];
        before += (g0 + i < w) ? t : 0u;
        all += t;
    }
    ex = before + x - v;
    tot = all;
}

// Per-byte carry of the leading bytes: bits 31..8 hold bytes 0..2 of a high
// word (most significant first), bits 0..2 flag which of them are defined.
// carry_op(a, b): b is later and wins where it is defined.
__device__ __forceinline__ uint32_t carry_op(uint32_t a, uint32_t b)
{
    const uint32_t sel = ((b & 1u) ? 0xFF000000u : 0u) | ((b & 2u) ? 0x00FF0000u : 0u) | ((b & 4u) ? 0x0000FF00u : 0u);
    return (b & sel) | (a & ~sel & 0xFFFFFF00u) | ((a | b) & 7u);
}

// exclusive carry scan over the group (identity 0)
template <int WPG>
__device__ __forceinline__ uint32_t gscan_carry(uint32_t v, uint32_t *slot)
{
    uint32_t x = v;
    x = carry_op(dpp0<0x111, 0xF>(x), x);
    x = carry_op(dpp0<0x112, 0xF>(x), x);
    x = carry_op(dpp0<0x114, 0xF>(x), x);
    x = carry_op(dpp0<0x118, 0xF>(x), x);
    x = carry_op(dpp0<0x142, 0xA>(x), x);
    x = carry_op(dpp0<0x143, 0xC>(x), x);
    uint32_t e = (uint32_t)__shfl_up((int)x, 1, 64);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) e = 0;
    if (lane == 63) slot[w] = x;
    lds_barrier();
    const int g0 = w - (w % WPG);
    uint32_t in = 0;
#pragma unroll
    for (int i = 0; i < WPG - 1; ++i)
        if (g0 + i < w) in = carry_op(in, slot[g0 + i]);
    return carry_op(in, e);
}

// Encoder scan: exclusive sums of (rp, cnt), totals of (bad, rp, cnt), and
// the last nonzero high word before this thread (flag f, value v).
template <int WPG>
__device__ __forceinline__ void gscan_enc(uint32_t bad, uint32_t rp, uint32_t cnt, uint32_t f, uint32_t v,
                                          uint32_t *slot, uint32_t &ex_rp, uint32_t &ex_cnt, uint32_t tot[3],
                                          uint32_t &in_f, uint32_t &in_v)
{
    uint32_t a = bad, b = rp, c = cnt;
#define QCZ_ENC_STEP(CTRL, RM)                                                   \
    {                                                                            \
        a += dpp0<CTRL, RM>(a);                                                  \
        b += dpp0<CTRL, RM>(b);                                                  \
        c += dpp0<CTRL, RM>(c);                                                  \
        const uint32_t yf = dpp0<CTRL, RM>(f), yv = dpp0<CTRL, RM>(v);           \
        v = f ? v : yv;                                                          \
        f |= yf;                                                                 \
    }
    QCZ_ENC_STEP(0x111, 0xF)
    QCZ_ENC_STEP(0x112, 0xF)
    QCZ_ENC_STEP(0x114, 0xF)
    QCZ_ENC_STEP(0x118, 0xF)
    QCZ_ENC_STEP(0x142, 0xA)
    QCZ_ENC_STEP(0x143, 0xC)
#undef QCZ_ENC_STEP
    uint32_t ef = (uint32_t)__shfl_up((int)f, 1, 64), ev = (uint32_t)__shfl_up((int)v, 1, 64);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) ef = 0;
    if (lane == 63) {
        slot[8 * w] = a;
        slot[8 * w + 1] = b;
        slot[8 * w + 2] = c;
        slot[8 * w + 3] = f;
        slot[8 * w + 4] = v;
    }
    lds_barrier();
    const int g0 = w - (w % WPG);
    uint32_t t0 = 0, t1 = 0, t2 = 0, b1 = 0, b2 = 0, pf = 0, pv = 0;
#pragma unroll
    for (int i = 0; i < WPG; ++i) {
        const uint32_t *q = slot + 8 * (g0 + i);
        const bool earlier = g0 + i < w;
        t0 += q[0];
        t1 += q[1];
        t2 += q[2];
        b1 += earlier ? q[1] : 0u;
        b2 += earlier ? q[2] : 0u;
        pv = (earlier && q[3]) ? q[4] : pv;
        pf |= earlier ? q[3] : 0u;
    }
    tot[0] = t0;
    tot[1] = t1;
    tot[2] = t2;
    ex_rp = b1 + b - rp;
    ex_cnt = b2 + c - cnt;
    in_f = ef ? ef : pf;
    in_v = ef ? ev : pv;
}

// ---------------------------------------------------------------------------
// entropy stage (header bit 5): the residual of a value (its bits after the
// leading bytes it shares with the previous value) is cut into 4-bit lanes;
// lane j covers bits [64-4j-w_j, 64-4j) of the value, w_j = min(4, K-4j),
// j < NN = ceil(K/4), and value i codes the lanes j >= 2 L_i.  Each lane is
// RAW (the w_j-bit symbol), CONST (one symbol, stored once) or CODED by a
// canonical Huffman code of at most 8 bits.  Sub-stream s holds the codes of
// positions 16s .. 16s+15; a 12-bit field per sub-stream gives its length.
// Kernels with the stage run C = 2048 doubles with two wavefronts per chunk,
// so thread lt owns positions 16 lt .. 16 lt + 15: exactly sub-stream lt.
// ---------------------------------------------------------------------------
constexpr uint32_t kHdrEnt = 0x20u;
// Solution D (Sec. 4.2): a PACK / SPARSE stream with header bit 6 stores its
// values re parts first, then im parts; stored position j holds interleaved
// position rsh_pos(j)
constexpr uint32_t kHdrRsh = 0x40u;
__device__ __forceinline__ int rsh_pos(int j, int C) { return j < C / 2 ? 2 * j : 2 * (j - C / 2) + 1; }

// The LDS copy of a chunk holds its values interleaved at vpos(i).  A thread's
// values in stored order (Solution D's when rsh) as (hi, lo) words, and whether
// one is subnormal; the two orders are separate loops (a uniform branch), so
// that the plain one reads at fixed offsets from the thread's first value.
template <int V>
__device__ __forceinline__ void load_stored(const double *vals, int first, int C, bool rsh, uint32_t (&xh)[V],
                                            uint32_t (&xl)[V], bool &sub)
{
    if (rsh) {
#pragma unroll
        for (int k = 0; k < V; ++k) {
            const uint64_t x = (uint64_t)__double_as_longlong(vals[vpos(rsh_pos(first + k, C))]);
            xh[k] = (uint32_t)(x >> 32);
            xl[k] = (uint32_t)x;
        }
    } else {
#pragma unroll
        for (int k = 0; k < V; ++k) {
            const uint64_t x = (uint64_t)__double_as_longlong(vals[vpos(first + k)]);
            xh[k] = (uint32_t)(x >> 32);
            xl[k] = (uint32_t)x;
        }
    }
#pragma unroll
    for (int k = 0; k < V; ++k) sub = sub || subnormal(xh[k], xl[k]);
}

// Values decoded in Solution D's stored order move to their interleaved
// positions (mine), or stay (plain streams), through the LDS copy.
template <int V>
__device__ __forceinline__ void store_interleaved(double *vals, int first, int C, bool mine, const double (&x)[V])
{
    if (mine) {
#pragma unroll
        for (int k = 0; k < V; ++k) vals[vpos(rsh_pos(first + k, C))] = x[k];
    } else {
#pragma unroll
        for (int k = 0; k < V; ++k) vals[vpos(first + k)] = x[k];
    }
}
constexpr int kEntMaxLen = 8;
constexpr int kEntSlotWords = 1024;   // per slot: decode tables (16 lanes x 256 bytes) or encode tables
enum { LANE_RAW = 0, LANE_CONST = 1, LANE_CODED = 2 };
// per slot in the entropy area: encode table (u16 per lane and symbol: code,
// bit-reversed, | length << 8) and lane records (4 words per lane)
constexpr int kEntRecWord0 = 128;

__device__ __forceinline__ int ent_lanes(int K) { return (K + 3) >> 2; }
__device__ __forceinline__ int ent_width(int K, int j)
{
    const int w = K - 4 * j;
    return w < 4 ? w : 4;
}
// lane j of a value (high word h, low word l)
__device__ __forceinline__ uint32_t ent_sym(uint32_t h, uint32_t l, int K, int j)
{
    const int w = ent_width(K, j);
    return j < 8 ? __builtin_amdgcn_ubfe(h, (uint32_t)(32 - 4 * j - w), (uint32_t)w)
                 : __builtin_amdgcn_ubfe(l, (uint32_t)(60 - 4 * j), 4u);
}
// table nibbles of a lane in mode m
__device__ __forceinline__ uint32_t ent_nibs(uint32_t m, int w) { return m == LANE_CONST ? 1u : m == LANE_CODED ? (1u << w) : 0u; }
// nibble k of a 64-bit word of sixteen 4-bit fields
__device__ __forceinline__ uint32_t nib64(uint64_t v, int k) { return (uint32_t)(v >> (4 * k)) & 15u; }

// one 4-bit field per bit of a 16-bit mask
__device__ __forceinline__ uint64_t spread16(uint32_t m)
{
    uint64_t x = m & 0xFFFFu;
    x = (x | (x << 24)) & 0x000000FF000000FFull;
    x = (x | (x << 12)) & 0x000F000F000F000Full;
    x = (x | (x << 6)) & 0x0303030303030303ull;
    x = (x | (x << 3)) & 0x1111111111111111ull;
    return x;
}

template <int N>
__device__ __forceinline__ void cswap(uint32_t (&k)[N], int a, int b)
{
    const uint32_t lo = min(k[a], k[b]), hi = max(k[a], k[b]);
    k[a] = lo;
    k[b] = hi;
}

// Code lengths of the lane's Huffman code (two or more symbols present; the
// counts are those of symbols 0..15).  Leaves in increasing (count, symbol)
// order (a bitonic sorting network on count << 4 | symbol), internal nodes
// in creation order as a second queue; each step joins the two lightest heads,
// the leaf first on equal weights.  Queue entries are weight << 16 | the mask
// of the leaves below (by sorted position) and live in this thread's LDS
// scratch q[32]; every merge adds one to the depth of the leaves below it.
// Lengths above 8 are cut to 8, then the longest code below 8 (fewest
// occurrences, then lowest symbol) grows by one bit while the Kraft sum
// exceeds 1.  Returns 16 four-bit lengths, symbol s at bits 4s.
__device__ uint64_t ent_huff_lengths(const uint32_t (&c)[16], uint32_t *q)
{
    uint32_t key[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) key[s] = c[s] ? (c[s] << 4) | (uint32_t)s : ~0u;
#pragma unroll
    for (int size = 2; size <= 16; size <<= 1)
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1)
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int jx = i ^ stride;
                if (jx > i) {
                    if ((i & size) == 0) cswap(key, i, jx);
                    else cswap(key, jx, i);
                }
            }
    int nl = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        nl += key[i] != ~0u ? 1 : 0;
        q[i] = key[i] != ~0u ? ((key[i] >> 4) << 16) | (1u << i) : ~0u;
    }
    uint32_t *node = q + 16;
    int h1 = 0, h2 = 0, nn = 0;
    uint64_t depth = 0;
    for (int it = 0; it < nl - 1; ++it) {
        const uint32_t lw0 = h1 < nl ? q[h1] : ~0u, lw1 = h1 + 1 < nl ? q[h1 + 1] : ~0u;
        const uint32_t nw0 = h2 < nn ? node[h2] : ~0u, nw1 = h2 + 1 < nn ? node[h2 + 1] : ~0u;
        const bool t1 = (lw0 >> 16) <= (nw0 >> 16);
        const uint32_t a = t1 ? lw0 : nw0;
        const uint32_t lh = t1 ? lw1 : lw0, nh = t1 ? nw0 : nw1;
        const bool t2 = (lh >> 16) <= (nh >> 16);
        const uint32_t bb = t2 ? lh : nh;
        h1 += (t1 ? 1 : 0) + (t2 ? 1 : 0);
        h2 += (t1 ? 0 : 1) + (t2 ? 0 : 1);
        const uint32_t m = (a | bb) & 0xFFFFu;
        node[nn++] = (((a >> 16) + (bb >> 16)) << 16) | m;
        depth += spread16(m);
    }
    uint64_t len = 0;
    uint32_t maxl = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const uint32_t d = nib64(depth, i);
        if (i < nl) len |= (uint64_t)d << (4 * (key[i] & 15u));
        maxl = (i < nl && d > maxl) ? d : maxl;
    }
    if (maxl > (uint32_t)kEntMaxLen) {
        uint32_t kraft = 0;
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            uint32_t l = nib64(len, s);
            if (l > (uint32_t)kEntMaxLen) {
                len = (len & ~(15ull << (4 * s))) | ((uint64_t)kEntMaxLen << (4 * s));
                l = kEntMaxLen;
            }
            kraft += l ? (1u << (kEntMaxLen - l)) : 0u;
        }
        while (kraft > (1u << kEntMaxLen)) {
            int best = -1;
            uint32_t bl = 0, bc = 0;
#pragma unroll
            for (int s = 0; s < 16; ++s) {
                const uint32_t l = nib64(len, s);
                const bool ok = l != 0 && l < (uint32_t)kEntMaxLen;
                const bool better = best < 0 || l > bl || (l == bl && c[s] < bc);
                if (ok && better) { best = s; bl = l; bc = c[s]; }
            }
            len += 1ull << (4 * best);
            kraft -= 1u << (kEntMaxLen - bl - 1);
        }
    }
    return len;
}

// Canonical code of symbol s (length l > 0) among the lengths `len`: symbols
// in increasing (length, symbol) order take consecutive codes, i.e. the code
// is the sum of 2^(8 - length) over the symbols before s, shifted down by
// 8 - l.
__device__ __forceinline__ uint32_t ent_canon_code(uint64_t len, int s, uint32_t l)
{
    uint32_t start = 0;
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        const uint32_t lt = nib64(len, t);
        const bool before = lt != 0 && (lt < l || (lt == l && t < s));
        start += before ? (1u << (kEntMaxLen - lt)) : 0u;
    }
    return start >> (kEntMaxLen - l);
}

// bit-reversed l-bit code (the code's first bit at the lowest position)
__device__ __forceinline__ uint32_t ent_rev(uint32_t code, uint32_t l)
{
    return l ? (__builtin_bitreverse32(code) >> (32u - l)) : 0u;
}

// Build lane j of the encoder's code from the slot's histogram hist[4][16][16]
// (four copies, summed): choose RAW / CONST / CODED by the format's rule, write
// the lane's encode table enc[16 * j + s] (u16: bit-reversed code | length << 8)
// and its record rec[4 j ..]: mode | symbol << 4 | table nibbles << 8, coded
// bits, lengths (low, high word).
__device__ __noinline__ void ent_build_lane(const uint32_t *hist, uint32_t *q, int K, int j, uint16_t *enc, uint32_t *rec)
{
    uint32_t c[16];
    uint32_t n = 0, distinct = 0, mx = 0, csym = 0;
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        c[s] = hist[(0 * 16 + j) * 16 + s] + hist[(1 * 16 + j) * 16 + s] + hist[(2 * 16 + j) * 16 + s] +
               hist[(3 * 16 + j) * 16 + s];
        n += c[s];
        distinct += c[s] ? 1u : 0u;
        mx = c[s] > mx ? c[s] : mx;
        csym = c[s] ? (uint32_t)s : csym;
    }
    const int w = ent_width(K, j);
    const uint32_t nsym = 1u << w, raw = n * (uint32_t)w;
    uint32_t mode = LANE_RAW, cost = raw;
    uint64_t len = 0;
    if (n > 0 && distinct == 1) {
        if (4u < raw) { mode = LANE_CONST; cost = 0; }
    } else if (distinct >= 2 && mx * nsym >= 2u * n) {
        len = ent_huff_lengths(c, q);
        uint32_t coded = 4u * nsym;
#pragma unroll
        for (int s = 0; s < 16; ++s) coded += c[s] * nib64(len, s);
        if (coded < raw) { mode = LANE_CODED; cost = coded - 4u * nsym; }
    }
    // canonical codes: the first code of each length follows from the number
    // of codes per length (8-bit fields, length l at bits 8(l-1)); symbols of
    // one length then take consecutive codes in symbol order
    uint64_t nx = 0;
    if (mode == LANE_CODED) {
        uint64_t cnt = 0;
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            const uint32_t l = nib64(len, s);
            cnt += l ? (1ull << (8u * (l - 1u))) : 0ull;
        }
        uint32_t code = 0;
#pragma unroll
        for (int l = 1; l <= kEntMaxLen; ++l) {
            if (l > 1) code = (code + (uint32_t)((cnt >> (8 * (l - 2))) & 0xFFu)) << 1;
            nx |= (uint64_t)(code & 0xFFu) << (8 * (l - 1));
        }
    }
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        uint32_t e = 0;
        if (mode == LANE_RAW) e = (uint32_t)s | ((uint32_t)w << 8);
        else if (mode == LANE_CODED) {
            const uint32_t l = nib64(len, s);
            if (l) {
                const uint32_t sh = 8u * (l - 1u);
                const uint32_t code = (uint32_t)(nx >> sh) & 0xFFu;
                nx += 1ull << sh;
                e = ent_rev(code, l) | (l << 8);
            }
        }
        enc[16 * j + s] = (uint16_t)e;
    }
    rec[4 * j] = mode | (csym << 4) | (ent_nibs(mode, w) << 8);
    rec[4 * j + 1] = cost;
    rec[4 * j + 2] = mode == LANE_CODED ? (uint32_t)len : 0u;
    rec[4 * j + 3] = mode == LANE_CODED ? (uint32_t)(len >> 32) : 0u;
}

// Decode tables of an entropy-coded stream: tab[256 j + x] = symbol | length
// << 4 for the next eight bits x of the stream (RAW: the low w bits; CONST:
// the symbol, length 0; CODED: the symbol whose bit-reversed code is x's low
// bits).  The caller has cleared tab (entries of a malformed stream may stay
// 0: a symbol 0 of length 0).  Thread lt fills the entries of (lane, symbol)
// pairs lt, lt + G, ...  tw0: first word of the table area; laneword: the
// stream's lane word.
template <int G>
__device__ void ent_fill_tables(const uint32_t *b, int tw0, uint32_t laneword, int K, uint8_t *tab, int lt)
{
    const int NN = ent_lanes(K);
    for (int p = lt; p < NN * 16; p += G) {
        const int j = p >> 4, s = p & 15;
        const int w = ent_width(K, j);
        const uint32_t mode = (laneword >> (2 * j)) & 3u;
        uint32_t off = 0;   // nibble offset of lane j in the table area
        for (int i = 0; i < j; ++i) off += ent_nibs((laneword >> (2 * i)) & 3u, ent_width(K, i));
        uint8_t *t = tab + 256 * j;
        if (mode == LANE_RAW) {
            if (s < (1 << w))
                for (int x = s; x < 256; x += 1 << w) t[x] = (uint8_t)(s | (w << 4));
        } else if (mode == LANE_CONST) {
            const uint32_t csym = __builtin_amdgcn_ubfe(b[clampw(tw0 + (int)(off >> 3))], 4u * (off & 7u), 4u);
            for (int x = 16 * s; x < 16 * s + 16; ++x) t[x] = (uint8_t)csym;
        } else if (mode == LANE_CODED && s < (1 << w)) {
            // the lane's 2^w lengths: nibbles off .. off + 2^w - 1
            const int wi = clampn<3>(tw0 + (int)(off >> 3));
            const uint32_t sh = 4u * (off & 7u);
            const uint64_t lo = ((uint64_t)b[wi + 1] << 32) | b[wi];
            uint64_t len = (lo >> sh) | (sh ? ((uint64_t)b[wi + 2] << (64 - sh)) : 0ull);
            if (w < 4) len &= (1ull << (4 << w)) - 1ull;
            const uint32_t l = nib64(len, s);
            if (l == 0 || l > (uint32_t)kEntMaxLen) continue;
            const uint32_t r = ent_rev(ent_canon_code(len, s, l), l);
            for (uint32_t x = r; x < 256u; x += 1u << l) t[x] = (uint8_t)(s | (l << 4));
        }
    }
}

// ---------------------------------------------------------------------------
// decode: the chunk staged in b[] -> the V values this thread owns
// ---------------------------------------------------------------------------
__device__ __forceinline__ int codes_word0(int mode, int C) { return mode == M_SPARSE ? 1 + ((C + 31) >> 5) : 1; }

// `hdr` is the stream header (an inactive slot passes a CONST2 header and
// active = false); `any_sparse` and `any_ent` (a slot holds an entropy-coded
// stream) are workgroup-uniform; etab is the slot's decode-table area.
// The residual fields of a thread's values (K < 64), from bit ob of the
// residual area bw: rd marks the values whose fields are read (stored and
// inside the buffer); each value gets its K-bit prefix bits below the shared
// leading bytes, and cbytes / cmin collect the carry-out of the leading-byte
// scan.  ALL: every value is read (a PACK stream), without per-value tests.
template <int V, bool ALL>
__device__ __forceinline__ void unpack_residuals(const uint32_t *bw, uint32_t ob, uint32_t rd, uint32_t stored,
                                                 uint32_t Lpos, uint32_t rtab, uint32_t up, uint32_t (&th)[V],
                                                 uint32_t (&tl)[V], uint32_t &cbytes, uint32_t &cmin)
{
    // four values at a time: their word pairs are read before any is used,
    // so one LDS round trip serves four values
    constexpr int U = V < 4 ? V : 4;
#pragma unroll
    for (int k0 = 0; k0 < V; k0 += U) {
        uint32_t lo[U], hi[U], sh[U], rr[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const int k = k0 + j;
            const uint32_t L = (Lpos >> (2 * k)) & 3u;
            rr[j] = (ALL || ((rd >> k) & 1u)) ? __builtin_amdgcn_ubfe(rtab, 8u * L, 8u) : 0u;
            const uint32_t wi = ob >> 5;
            lo[j] = bw[wi];
            hi[j] = bw[wi + 1];
            sh[j] = ob & 31u;
            ob += rr[j];
        }
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const int k = k0 + j;
            const uint32_t L = (Lpos >> (2 * k)) & 3u;
            // lossy levels keep at most 29 bits, so rr < 32
            const uint32_t p = (fshr(hi[j], lo[j], sh[j]) & ((1u << rr[j]) - 1u)) << up;
            th[k] = p;
            tl[k] = 0u;
            const uint32_t Ls = (ALL || ((stored >> k) & 1u)) ? L : 3u;
            const uint32_t own = (~0u >> (8u * Ls)) & 0xFFFFFF00u;
            cbytes = (own & p) | (~own & cbytes);
            cmin = Ls < cmin ? Ls : cmin;
        }
    }
}

template <int V, int WPG, bool ENT = false>
__device__ void decode_group(const uint32_t *b, uint32_t hdr, bool active, bool any_sparse, int C, int lt,
                             uint32_t *slotA, uint32_t *slotB, uint32_t *slotC, uint32_t (&th)[V], uint32_t (&tl)[V],
                             bool any_ent = false, uint8_t *etab = nullptr)
{
    static_assert(!ENT || V == 16, "the entropy stage runs one sub-stream of 16 values per thread");
    const int mode = (int)(hdr & 3u);
    int lev = (int)((hdr >> 2) & 7u);
    if (lev >= kLevels) lev = 0;
    const int K = sig_bits(lev);
    const int first = lt * V;
    const uint32_t vmask = (V >= 32) ? ~0u : ((1u << V) - 1u);
    uint32_t stored = 0;
    if (mode == M_PACK) stored = vmask;
    else if (mode == M_SPARSE) stored = (b[clampw(1 + (first >> 5))] >> (first & 31)) & vmask;
    uint32_t rank0 = (uint32_t)first, nnz = (uint32_t)C;
    if (any_sparse) {
        uint32_t ex, tot;
        gscan_add<WPG>(__popc(stored), slotA, ex, tot);
        if (mode == M_SPARSE) { rank0 = ex; nnz = tot; }
    }
    const int cw0 = codes_word0(mode, C);
    const int res_w0 = cw0 + (int)((nnz + 15u) >> 4);
    const uint32_t cbit = 2u * rank0;
    const int cwi = clampn<2>(cw0 + (int)(cbit >> 5));
    const uint32_t cw = fshr(b[cwi + 1], b[cwi], cbit & 31u);

    // codes by position (a SPARSE chunk's codes are in rank order; wave-uniform branch)
    uint32_t Lpos = 0, rsum = 0;
    if (mode == M_SPARSE) {
        // spread the rank-ordered codes to the stored positions
        uint32_t j2 = 0;   // two bits per code already taken
#pragma unroll
        for (int k = 0; k < V; ++k) {
            const uint32_t st = (stored >> k) & 1u;
            const uint32_t L = __builtin_amdgcn_ubfe(cw, j2 & 31u, 2u);
            Lpos |= (st ? L : 0u) << (2 * k);
            j2 += 2u * st;
        }
        rsum = resid_total(Lpos, K, (uint32_t)__popc(stored));   // zero codes at empty positions add nothing
    } else if (stored) {
        Lpos = (V >= 16) ? cw : (cw & ((1u << (2 * V)) - 1u));
        rsum = resid_total(Lpos, K, (uint32_t)V);
    }
    // entropy-coded stream: decode tables of its lanes, and my sub-stream's
    // bit length (field lt of the length area) in place of the residual total
    const bool my_ent = ENT && active && (hdr & kHdrEnt) != 0 && mode != M_CONST2;
    int bw0 = 0;   // first word of the entropy-coded bit stream
    if (ENT && any_ent) {
        const int NN = ent_lanes(K);
        const uint32_t lw = my_ent ? b[clampw(res_w0)] : 0u;
        uint32_t *tw = reinterpret_cast<uint32_t *>(etab);
        if (my_ent)
            for (int i = lt; i < 64 * NN; i += 64 * WPG) tw[i] = 0u;
        lds_barrier();
        if (my_ent) ent_fill_tables<64 * WPG>(b, res_w0 + 1, lw, K, etab, lt);
        lds_barrier();
        if (my_ent) {
            uint32_t nib = 0;
            for (int j = 0; j < NN; ++j) nib += ent_nibs((lw >> (2 * j)) & 3u, ent_width(K, j));
            const int sw0 = res_w0 + 1 + (int)((nib + 7u) >> 3);
            const uint32_t bit = 12u * (uint32_t)lt;
            const int wi = clampn<2>(sw0 + (int)(bit >> 5));
            rsum = fshr(b[wi + 1], b[wi], bit & 31u) & 0xFFFu;
            bw0 = sw0 + ((12 * (C / 16) + 31) >> 5);
        }
    }
    uint32_t o, rtot;
    gscan_add<WPG>(rsum, slotB, o, rtot);

    // carry-out of my values for the leading-byte scan: the top three bytes
    // as last defined by one of my stored values (a value with L shared
    // leading bytes defines the 3 - L after them) and the smallest such L
    uint32_t cbytes = 0, cmin = 3;
    if (ENT && my_ent) {
        // my sub-stream: for each stored value the lanes 2L .. NN-1, each an
        // eight-bit table lookup on a bit window refilled a word at a time
        const int NN = ent_lanes(K);
        const int wi = bw0 + (int)(o >> 5);
        const uint32_t sh = o & 31u;
        uint64_t win = (((uint64_t)b[clampw(wi + 1)] << 32) | b[clampw(wi)]) >> sh;
        int avail = 64 - (int)sh;
        int nextw = wi + 2;
#pragma unroll
        for (int k = 0; k < V; ++k) {
            const uint32_t st = (stored >> k) & 1u;
            const uint32_t L = (Lpos >> (2 * k)) & 3u;
            uint32_t vh = 0, vl = 0;
            const int j0 = st ? 2 * (int)L : NN;
            for (int j = j0; j < NN; ++j) {
                if (avail < 8) {
                    win |= (uint64_t)b[clampw(nextw)] << avail;
                    ++nextw;
                    avail += 32;
                }
                const uint32_t e = etab[256 * j + (uint32_t)(win & 255u)];
                const uint32_t sym = e & 15u, l = e >> 4;
                win >>= l;
                avail -= (int)l;
                if (j < 8) vh |= sym << (32 - 4 * j - ent_width(K, j));
                else vl |= sym << (60 - 4 * j);
            }
            th[k] = vh;
            tl[k] = vl;
            const uint32_t Ls = st ? L : 3u;
            const uint32_t own = (~0u >> (8u * Ls)) & 0xFFFFFF00u;
            cbytes = (own & vh) | (~own & cbytes);
            cmin = Ls < cmin ? Ls : cmin;
        }
    } else if (K < 64) {
        const uint32_t up = (uint32_t)(32 - K);
        // residual width of each code, one byte apiece
        const uint32_t rtab = resid_bits(K, 0) | (resid_bits(K, 1) << 8) | (resid_bits(K, 2) << 16) |
                              (resid_bits(K, 3) << 24);
        // my fields lie in [o, o + rsum) past the first residual word; a valid
        // stream keeps them inside the buffer, a corrupt one reads empty fields
        const bool fits = res_w0 + (int)((o + rsum) >> 5) <= kBufWords - 2;
        const uint32_t rd = fits ? stored : 0u;
        const uint32_t ob = fits ? o : 0u;
        if (rd == vmask)   // every value stored and inside the buffer (PACK)
            unpack_residuals<V, true>(b + res_w0, ob, rd, stored, Lpos, rtab, up, th, tl, cbytes, cmin);
        else
            unpack_residuals<V, false>(b + res_w0, ob, rd, stored, Lpos, rtab, up, th, tl, cbytes, cmin);
    } else {
#pragma unroll
        for (int k = 0; k < V; ++k) {
            const uint32_t st = (stored >> k) & 1u;
            const uint32_t L = (Lpos >> (2 * k)) & 3u;
            const uint32_t r = st ? 64u - 8u * L : 0u;
            const int wi = clampn<3>(res_w0 + (int)(o >> 5));
            const uint32_t w0 = b[wi], w1 = b[wi + 1], w2 = b[wi + 2];
            const uint32_t Rl = r ? fshr(w1, w0, o & 31u) : 0u;
            const uint32_t Rh = fshr(w2, w1, o & 31u) & (r ? low_mask32(r - 32u) : 0u);
            o += r;
            th[k] = Rh;
            tl[k] = Rl;
            const uint32_t Ls = st ? L : 3u;
            const uint32_t own = (~0u >> (8u * Ls)) & 0xFFFFFF00u;
            cbytes = (own & Rh) | (~own & cbytes);
            cmin = Ls < cmin ? Ls : cmin;
        }
    }
    // (low three bits: which of the three bytes are defined, top byte first)
    const uint32_t carry = cbytes | ((7u << cmin) & 7u);
    // the value before the chunk is 0: every leading byte defined as zero
    uint32_t prev = carry_op(7u, gscan_carry<WPG>(carry, slotC)) & 0xFFFFFF00u;
    if (mode == M_CONST2) {
        const uint32_t c0l = active ? b[1] : 0u, c0h = active ? b[2] : 0u;
        const uint32_t c1l = active ? b[3] : 0u, c1h = active ? b[4] : 0u;
#pragma unroll
        for (int k = 0; k < V; ++k) {
            const bool odd = ((first + k) & 1) != 0;
            th[k] = odd ? c1h : c0h;
            tl[k] = odd ? c1l : c0l;
        }
    } else if (stored == vmask) {
        // every value stored (PACK): each one is the previous value for the next
#pragma unroll
        for (int k = 0; k < V; ++k) {
            const uint32_t mine = ~0u >> (8u * ((Lpos >> (2 * k)) & 3u));
            prev = (mine & th[k]) | (~mine & prev);
            th[k] = prev;
        }
    } else {
#pragma unroll
        for (int k = 0; k < V; ++k) {
            const uint32_t st = (stored >> k) & 1u;
            // the L leading bytes shared with the previous value, the rest mine
            // (an empty position has code 0 and zero words, so it stays zero)
            const uint32_t mine = ~0u >> (8u * ((Lpos >> (2 * k)) & 3u));
            const uint32_t v = (mine & th[k]) | (~mine & prev);
            th[k] = v;
            prev = st ? v : prev;
        }
    }
}

// ---------------------------------------------------------------------------
// encode
// ---------------------------------------------------------------------------
template <int V>
struct EncPlan {
    uint32_t th[V], tl[V];  // truncated values
    uint32_t codes;         // PACK codes by position (2 bits each)
    uint32_t scodes;        // SPARSE codes of my nonzero values, rank order
    uint32_t nzm;           // my nonzero positions
    uint32_t pack_off;      // bit offset of my PACK residuals
    uint32_t sp_off;        // bit offset of my SPARSE residuals
    uint32_t rank0;         // rank of my first nonzero value
    uint32_t nnz;
    uint32_t c0h, c0l, c1h, c1l;  // values 0 and 1 (CONST2)
    int mode, lev, K;
    uint32_t size;
    bool ent;               // the body's residuals are entropy-coded
    bool rsh;               // values stored re parts first (Solution D; never on CONST2)
    uint32_t ent_off;       // bit offset of my sub-stream in the entropy-coded bit stream
    uint32_t ent_bits;      // its length
    uint32_t laneword;      // lane modes (2 bits per lane)
};

// the stored values a thread codes (PACK: all, SPARSE: the nonzero ones) and
// their two-bit codes (PACK: by position, SPARSE: in rank order)
template <int V>
__device__ __forceinline__ void ent_values(const EncPlan<V> &e, uint32_t &mask, uint32_t &codes, bool &sparse)
{
    const uint32_t vmask = (V >= 32) ? ~0u : ((1u << V) - 1u);
    sparse = e.mode == M_SPARSE;
    mask = e.mode == M_CONST2 ? 0u : (sparse ? e.nzm : vmask);
    codes = sparse ? e.scodes : e.codes;
}

// Entropy stage of the plan (ENT kernels, ent_on uniform over the launch).
// The entropy helpers are called, not inlined (ent_plan, ent_emit,
// ent_build_lane): inlined into the job kernel at three workgroups per CU,
// the plan came out wrong (tests/test_gpu_entropy.py), called it is exact
// and its registers stay out of the kernel's allocation.
// lane histograms (four copies, by lane & 3, in the slot's buffer b, free
// once the plan's scans have passed), one builder thread per lane, the size
// of the entropy-coded body from the lanes' costs, and each thread's bit
// offset.  Contains barriers: every thread calls it.
template <int V, int WPG>
__device__ __noinline__ void ent_plan(EncPlan<V> &e, int C, int lt, uint32_t *b, uint32_t *ent, uint32_t *slot)
{
    constexpr int G = 64 * WPG;
    const int K = e.K, NN = ent_lanes(K);
    uint32_t mask, codes;
    bool sparse;
    ent_values<V>(e, mask, codes, sparse);
    uint32_t *hist = b;
    for (int i = lt; i < 1024; i += G) hist[i] = 0u;
    lds_barrier();
    const uint32_t rep = threadIdx.x & 3u;
    {
        uint32_t j2 = 0;
#pragma unroll
        for (int k = 0; k < V; ++k) {
            const bool on = ((mask >> k) & 1u) != 0;
            const uint32_t L = __builtin_amdgcn_ubfe(codes, sparse ? (j2 & 31u) : 2u * k, 2u);
            j2 += on ? 2u : 0u;
            for (int j = on ? 2 * (int)L : NN; j < NN; ++j)
                atomicAdd(&hist[(rep * 16u + (uint32_t)j) * 16u + ent_sym(e.th[k], e.tl[k], K, j)], 1u);
        }
    }
    lds_barrier();
    uint16_t *enc = reinterpret_cast<uint16_t *>(ent);
    uint32_t *rec = ent + kEntRecWord0;
    if (lt < NN) ent_build_lane(hist, b + 1024 + 32 * lt, K, lt, enc, rec);
    lds_barrier();
    uint32_t bits = 0, nibs = 0, lw = 0;
    for (int j = 0; j < NN; ++j) {
        const uint32_t r0 = rec[4 * j];
        bits += rec[4 * j + 1];
        nibs += r0 >> 8;
        lw |= (r0 & 3u) << (2 * j);
    }
    const uint32_t N = sparse ? e.nnz : (uint32_t)C;
    const uint32_t lead = sparse ? 4u + 4u * (uint32_t)((C + 31) / 32) : 4u;
    const uint32_t esize = lead + 4u * ((N + 15u) / 16u) + 4u + 4u * ((nibs + 7u) / 8u) +
                           4u * ((12u * (uint32_t)(C / 16) + 31u) / 32u) + (bits + 7u) / 8u;
    const bool take = e.mode != M_CONST2 && esize < e.size;
    uint32_t mine = 0;
    if (take) {
        uint32_t j2 = 0;
#pragma unroll
        for (int k = 0; k < V; ++k) {
            const bool on = ((mask >> k) & 1u) != 0;
            const uint32_t L = __builtin_amdgcn_ubfe(codes, sparse ? (j2 & 31u) : 2u * k, 2u);
            j2 += on ? 2u : 0u;
            for (int j = on ? 2 * (int)L : NN; j < NN; ++j)
                mine += (uint32_t)enc[16 * j + ent_sym(e.th[k], e.tl[k], K, j)] >> 8;
        }
    }
    uint32_t tot;
    gscan_add<WPG>(mine, slot, e.ent_off, tot);
    e.ent = take;
    e.ent_bits = mine;
    e.laneword = lw;
    if (take) e.size = esize;
}

// Plan the stream of one chunk.  x: my values (hi, lo); xprev_hi: high word of
// the value before mine; x0/x1: values 0 and 1 of the chunk.  `sub` is the
// group's subnormal flag.  Contains barriers: every thread calls it; the plan
// of a group with no chunk (stale values) is computed and ignored.
// The per-value part of the plan: truncated words, CONST2 test bits, codes,
// nonzero positions and the last nonzero high word.  LOSSLESS is a template
// argument so that the lossy instance (low words all zero, as are the CONST2
// references' low words) spends no instructions on low words.
template <int V, bool LOSSLESS>
__device__ __forceinline__ void plan_values(const uint32_t (&xh)[V], const uint32_t (&xl)[V], uint32_t mh,
                                            uint32_t prev, int first, uint32_t re_h, uint32_t re_l, uint32_t im_h,
                                            uint32_t im_l, EncPlan<V> &e, uint32_t &badbits, uint32_t &codes,
                                            uint32_t &nzm, uint32_t &lv)
{
#pragma unroll
    for (int k = 0; k < V; ++k) {
        const uint32_t h = xh[k] & mh;
        const uint32_t l = LOSSLESS ? xl[k] : 0u;
        e.th[k] = h;
        e.tl[k] = l;
        const bool odd = ((first + k) & 1) != 0;
        const uint32_t dh = h ^ (odd ? im_h : re_h);   // differs from value 0 / 1
        badbits |= LOSSLESS ? (dh | (l ^ (odd ? im_l : re_l))) : dh;
        const uint32_t L = lead_bytes(h, prev);
        codes |= L << (2 * k);
        prev = h;
        const bool nz = (LOSSLESS ? (h | l) : h) != 0;
        nzm |= nz ? (1u << k) : 0u;
        lv = nz ? h : lv;
    }
}

template <int V, int WPG, bool ENT = false>
__device__ void encode_plan(const uint32_t (&xh)[V], const uint32_t (&xl)[V], uint32_t xprev_hi, uint64_t x0,
                            uint64_t x1, int lev_req, bool sub, int C, int lt, uint32_t *slotB,
                            uint32_t *slotC, EncPlan<V> &e, bool ent_on = false, uint32_t *b = nullptr,
                            uint32_t *ent = nullptr, uint32_t *slotD = nullptr, bool rsh = false)
{
    const int first = lt * V;
    const int lev = sub ? 0 : lev_req;  // a chunk with a subnormal is kept lossless
    const int K = sig_bits(lev);
    const uint32_t mh = sig_mask_hi(K);
    const bool lossless = K >= 64;
    e.c0h = (uint32_t)(x0 >> 32) & mh;
    e.c0l = lossless ? (uint32_t)x0 : 0u;
    e.c1h = (uint32_t)(x1 >> 32) & mh;
    e.c1l = lossless ? (uint32_t)x1 : 0u;

    uint32_t badbits = 0, nzm = 0, codes = 0, lf = 0, lv = 0;
    uint32_t prev = xprev_hi & mh;
    // CONST2 test: value k of mine is compared with value 0 (a real part) or
    // value 1 (an imaginary part).  Interleaved, that follows the parity of its
    // position; in Solution D's order a thread's values all lie in one half, so
    // both references are that half's
    const uint32_t half_h = first >= C / 2 ? e.c1h : e.c0h, half_l = first >= C / 2 ? e.c1l : e.c0l;
    const uint32_t re_h = rsh ? half_h : e.c0h, re_l = rsh ? half_l : e.c0l;
    const uint32_t im_h = rsh ? half_h : e.c1h, im_l = rsh ? half_l : e.c1l;
    if (lossless)
        plan_values<V, true>(xh, xl, mh, prev, first, re_h, re_l, im_h, im_l, e, badbits, codes, nzm, lv);
    else
        plan_values<V, false>(xh, xl, mh, prev, first, re_h, re_l, im_h, im_l, e, badbits, codes, nzm, lv);
    const uint32_t cnt = __popc(nzm);
    lf = nzm ? 1u : 0u;
    const uint32_t bad = badbits ? 1u : 0u;
    const uint32_t rp = resid_total(codes, K, (uint32_t)V);
    uint32_t tot[3], in_f, in_v;
    gscan_enc<WPG>(bad, rp, cnt, lf, lv, slotB, e.pack_off, e.rank0, tot, in_f, in_v);
    const bool const2 = tot[0] == 0;
    const uint32_t RP = tot[1], NNZ = tot[2];
    e.nnz = NNZ;
    // SPARSE can only win when the chunk has zeros; with none its body equals
    // PACK's plus the bitmap.  The decision must be uniform over the workgroup:
    // the scan runs when any slot (WPG wavefronts each) needs it.
    const int w = threadIdx.x >> 6;
    const int g0 = w - (w % WPG);   // my slot's first wavefront
    const int nw = (int)(blockDim.x >> 6);
    bool need_other = false;
    for (int o0 = 0; o0 < nw; o0 += WPG) {
        if (o0 == g0) continue;
        uint32_t other_bad = 0, other_nnz = 0;
#pragma unroll
        for (int i = 0; i < WPG; ++i) {
            other_bad += slotB[8 * (o0 + i)];
            other_nnz += slotB[8 * (o0 + i) + 2];
        }
        need_other = need_other || (other_bad != 0 && other_nnz < (uint32_t)C);
    }
    const bool need_me = !const2 && NNZ < (uint32_t)C;
    uint32_t RS = 0;
    e.scodes = 0;
    e.sp_off = 0;
    if (need_me || need_other) {
        // (the scan has a barrier: both slots take part when either needs it)
        uint32_t rs = 0;
        if (need_me) {
            uint32_t sprev = in_f ? in_v : 0u;
            uint32_t scodes = 0, j2 = 0;
#pragma unroll
            for (int k = 0; k < V; ++k) {
                const bool nz = ((nzm >> k) & 1u) != 0;
                const uint32_t L = lead_bytes(e.th[k], sprev);
                scodes |= nz ? (L << (j2 & 31u)) : 0u;
                j2 += nz ? 2u : 0u;
                sprev = nz ? e.th[k] : sprev;
            }
            e.scodes = scodes;
            rs = resid_total(scodes, K, cnt);
        }
        gscan_add<WPG>(rs, slotC, e.sp_off, RS);
    }
    const uint32_t pack_size = 4u + 4u * (uint32_t)((C + 15) / 16) + (RP + 7u) / 8u;
    const uint32_t sparse_size = 4u + 4u * (uint32_t)((C + 31) / 32) + 4u * ((NNZ + 15u) / 16u) + (RS + 7u) / 8u;
    e.codes = codes;
    e.nzm = nzm;
    e.lev = lev;
    e.K = K;
    e.rsh = rsh && !const2;
    if (const2) { e.mode = M_CONST2; e.size = 20; }
    else if (need_me && sparse_size < pack_size) { e.mode = M_SPARSE; e.size = sparse_size; }
    else { e.mode = M_PACK; e.size = pack_size; }
    e.ent = false;
    e.ent_off = e.ent_bits = e.laneword = 0;
    if (ENT && ent_on) ent_plan<V, WPG>(e, C, lt, b, ent, slotD);
}

// OR an r-bit field (r <= 32) into the word stream at bit offset o
__device__ __forceinline__ void or_bits32(uint32_t *b, int base, uint32_t o, uint32_t R, uint32_t r)
{
    if (r == 0) return;
    const uint64_t x = (uint64_t)R << (o & 31u);
    const int wi = base + (int)(o >> 5);
    atomicOr(&b[clampw(wi)], (uint32_t)x);
    if ((uint32_t)(x >> 32)) atomicOr(&b[clampw(wi + 1)], (uint32_t)(x >> 32));
}

// OR a 64-bit field (Rh:Rl, r bits, 32 < r <= 64) into the stream
__device__ __forceinline__ void or_bits64(uint32_t *b, int base, uint32_t o, uint32_t Rh, uint32_t Rl)
{
    const uint32_t sh = o & 31u;
    const uint64_t xl = (uint64_t)Rl << sh, xh = (uint64_t)Rh << sh;
    const int wi = base + (int)(o >> 5);
    atomicOr(&b[clampw(wi)], (uint32_t)xl);
    atomicOr(&b[clampw(wi + 1)], (uint32_t)(xl >> 32) | (uint32_t)xh);
    if ((uint32_t)(xh >> 32)) atomicOr(&b[clampw(wi + 2)], (uint32_t)(xh >> 32));
}

// residual field of a value: the low r bits of its K-bit significant prefix
// (SPARSE a template argument: the PACK instance tests nothing per value)
template <int V, bool SPARSE>
__device__ __forceinline__ void emit_residuals(uint32_t *b, int base, uint32_t o, const EncPlan<V> &e,
                                               uint32_t mask, uint32_t codes)
{
    constexpr bool sparse = SPARSE;
    const int K = e.K;
    uint32_t j2 = 0;   // two bits per code of the values emitted so far (SPARSE: rank order)
    if (K < 64) {
        // a thread's fields are contiguous: assemble them in a 64-bit
        // accumulator and OR each word into the zeroed stream as it fills (the
        // first word is shared with the thread before, the last partial one
        // with the thread after; the others are mine alone)
        // (the planned size bounds every word index: no clamping)
        const uint32_t rtab = resid_bits(K, 0) | (resid_bits(K, 1) << 8) | (resid_bits(K, 2) << 16) |
                              (resid_bits(K, 3) << 24);
        uint64_t acc = 0;
        uint32_t nb = o & 31u;
        int wi = base + (int)(o >> 5);
#pragma unroll
        for (int k = 0; k < V; ++k) {
            const bool on = ((mask >> k) & 1u) != 0;
            const uint32_t L = __builtin_amdgcn_ubfe(codes, sparse ? (j2 & 31u) : 2u * k, 2u);
            j2 += on ? 2u : 0u;
            const uint32_t r = on ? __builtin_amdgcn_ubfe(rtab, 8u * L, 8u) : 0u;   // < 32 at every lossy level
            acc |= (uint64_t)__builtin_amdgcn_ubfe(e.th[k], (uint32_t)(32 - K), r) << nb;   // r bits from bit 32 - K
            nb += r;
            if (nb >= 32u) {
                atomicOr(&b[wi], (uint32_t)acc);
                ++wi;
                acc >>= 32;
                nb -= 32u;
            }
        }
        if (nb > 0u) atomicOr(&b[wi], (uint32_t)acc);
        return;
    }
#pragma unroll
    for (int k = 0; k < V; ++k) {
        const bool on = ((mask >> k) & 1u) != 0;
        const uint32_t L = __builtin_amdgcn_ubfe(codes, sparse ? (j2 & 31u) : 2u * k, 2u);
        j2 += on ? 2u : 0u;
        if (on) {
            const uint32_t r = 64u - 8u * L;
            or_bits64(b, base, o, e.th[k] & (~0u >> (8u * L)), e.tl[k]);
            o += r;
        }
    }
}

// OR a field of r <= 64 bits into the word stream at bit offset o
__device__ __forceinline__ void or_field(uint32_t *b, int base, uint32_t o, uint64_t v, uint32_t r)
{
    if (r == 0) return;
    const uint32_t sh = o & 31u;
    const int wi = base + (int)(o >> 5);
    const uint64_t lo = v << sh;
    atomicOr(&b[clampw(wi)], (uint32_t)lo);
    if ((uint32_t)(lo >> 32)) atomicOr(&b[clampw(wi + 1)], (uint32_t)(lo >> 32));
    if (sh + r > 64u) atomicOr(&b[clampw(wi + 2)], (uint32_t)(v >> (64u - sh)));
}

// entropy-coded body after the codes area (word ew0): lane word, table
// nibbles (lane builders), my sub-stream's length field and my codes
template <int V>
__device__ __noinline__ void ent_emit(uint32_t *b, const EncPlan<V> &e, int C, int lt, int ew0, const uint32_t *ent)
{
    const int K = e.K, NN = ent_lanes(K);
    const uint16_t *enc = reinterpret_cast<const uint16_t *>(ent);
    const uint32_t *rec = ent + kEntRecWord0;
    uint32_t nibs = 0, off = 0;
    for (int j = 0; j < NN; ++j) {
        const uint32_t n = rec[4 * j] >> 8;
        off += j < lt ? n : 0u;
        nibs += n;
    }
    if (lt == 0) b[ew0] = e.laneword;
    if (lt < NN) {
        const uint32_t r0 = rec[4 * lt];
        const uint32_t n = r0 >> 8;
        const uint64_t v = (r0 & 3u) == LANE_CONST ? (uint64_t)((r0 >> 4) & 15u)
                                                    : (((uint64_t)rec[4 * lt + 3] << 32) | rec[4 * lt + 2]);
        or_field(b, ew0 + 1, 4u * off, v, 4u * n);
    }
    const int sw0 = ew0 + 1 + (int)((nibs + 7u) >> 3);
    or_field(b, sw0, 12u * (uint32_t)lt, e.ent_bits, 12u);
    const int bw0 = sw0 + ((12 * (C / 16) + 31) >> 5);
    uint32_t mask, codes;
    bool sparse;
    ent_values<V>(e, mask, codes, sparse);
    uint64_t acc = 0;
    uint32_t nb = e.ent_off & 31u;
    int wi = bw0 + (int)(e.ent_off >> 5);
    bool first = true;
    uint32_t j2 = 0;
#pragma unroll
    for (int k = 0; k < V; ++k) {
        const bool on = ((mask >> k) & 1u) != 0;
        const uint32_t L = __builtin_amdgcn_ubfe(codes, sparse ? (j2 & 31u) : 2u * k, 2u);
        j2 += on ? 2u : 0u;
        for (int j = on ? 2 * (int)L : NN; j < NN; ++j) {
            const uint32_t x = enc[16 * j + ent_sym(e.th[k], e.tl[k], K, j)];
            acc |= (uint64_t)(x & 0xFFu) << nb;
            nb += x >> 8;
            if (nb >= 32u) {
                if (first) atomicOr(&b[clampw(wi)], (uint32_t)acc);
                else b[clampw(wi)] = (uint32_t)acc;
                first = false;
                ++wi;
                acc >>= 32;
                nb -= 32u;
            }
        }
    }
    if (nb > 0u) atomicOr(&b[clampw(wi)], (uint32_t)acc);
}

// write the planned stream into b[] (already zeroed); no barriers inside
template <int V>
__device__ void encode_emit(uint32_t *b, const EncPlan<V> &e, int C, int lt, const uint32_t *ent = nullptr)
{
    const int first = lt * V;
    if (lt == 0) b[0] = (uint32_t)e.mode | ((uint32_t)e.lev << 2) | (e.ent ? kHdrEnt : 0u) | (e.rsh ? kHdrRsh : 0u);
    if (e.mode == M_CONST2) {
        if (lt == 0) {
            b[1] = e.c0l; b[2] = e.c0h;
            b[3] = e.c1l; b[4] = e.c1h;
        }
        return;
    }
    const uint32_t vmask = (V >= 32) ? ~0u : ((1u << V) - 1u);
    if (e.mode == M_PACK) {
        const uint32_t bit = 2u * (uint32_t)first;
        if (V == 16) b[1 + (bit >> 5)] = e.codes;
        else atomicOr(&b[1 + (bit >> 5)], e.codes << (bit & 31));
        if (e.ent) ent_emit<V>(b, e, C, lt, 1 + C / 16, ent);
        else emit_residuals<V, false>(b, 1 + C / 16, e.pack_off, e, vmask, e.codes);
    } else {  // M_SPARSE
        if (e.nzm) atomicOr(&b[1 + (first >> 5)], e.nzm << (first & 31));
        const int cw0 = 1 + ((C + 31) >> 5);
        const uint32_t cnt = __popc(e.nzm);
        if (cnt) {
            const uint32_t bit = 2u * e.rank0;
            const uint64_t v = (uint64_t)e.scodes << (bit & 31);
            const int wi = cw0 + (int)(bit >> 5);
            if ((uint32_t)v) atomicOr(&b[clampw(wi)], (uint32_t)v);
            if ((uint32_t)(v >> 32)) atomicOr(&b[clampw(wi + 1)], (uint32_t)(v >> 32));
        }
        if (e.ent) ent_emit<V>(b, e, C, lt, cw0 + (int)((e.nnz + 15u) >> 4), ent);
        else emit_residuals<V, true>(b, cw0 + (int)((e.nnz + 15u) >> 4), e.sp_off, e, e.nzm, e.scodes);
    }
}

// ---------------------------------------------------------------------------
// gates: Eq. (6) on pairs, Eq. (7) with controls, diagonal phases, X, MCZ.
// Fixed FMA order so results are reproducible to the bit.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void lin2(double ur, double ui, double vr, double vi, double ar, double ai,
                                     double br, double bi, double &yr, double &yi)
{
    yr = __fma_rn(vr, br, __fma_rn(-vi, bi, __fma_rn(ur, ar, -(ui * ai))));
    yi = __fma_rn(vr, bi, __fma_rn(vi, br, __fma_rn(ur, ai, ui * ar)));
}

__device__ __forceinline__ void dmul(double dr, double di, double ar, double ai, double &yr, double &yi)
{
    yr = __fma_rn(dr, ar, -(di * ai));
    yi = __fma_rn(dr, ai, di * ar);
}

__device__ __forceinline__ bool unit_phase(double re, double im) { return re == 1.0 && im == 0.0; }

// phase idx (0..3) of a diagonal gate; m is the workgroup's LDS copy of the
// gate parameters (an indexed read of the kernel arguments would be a memory
// load, and its wait would cover every outstanding memory access)
__device__ __forceinline__ void phase_of(const double *m, int idx, double &pr, double &pi)
{
    pr = m[2 * idx];
    pi = m[2 * idx + 1];
}

// a diagonal gate leaves chunk c alone when every phase reachable in it is 1
// unit_mask: bit idx set when phase idx is 1 (computed once per launch)
template <class D>
__device__ bool diag_touches(const D &gd, uint32_t unit_mask, uint64_t c, int cb)
{
    const int nidx = gd.kind == K_DIAG1 ? 2 : 4;
#pragma unroll
    for (int idx = 0; idx < 4; ++idx) {
        if (idx >= nidx) break;
        int b1 = idx & 1, b2 = idx >> 1;
        if (gd.q >= cb && (int)((c >> (gd.q - cb)) & 1ull) != b1) continue;
        if (gd.kind == K_DIAG2 && gd.q2 >= cb && (int)((c >> (gd.q2 - cb)) & 1ull) != b2) continue;
        if (!((unit_mask >> idx) & 1u)) return true;
    }
    return false;
}

__device__ __forceinline__ uint64_t deposit(const GateDesc &gd, uint64_t k)
{
    // k's bits fill the chunk-index positions outside fixed_mask in order:
    // open a hole at every fixed position, lowest first, then set the fixed
    // values (a loop over the few fixed bits, not over all index bits)
    uint64_t c = k;
    uint64_t fm = gd.fixed_mask;
    while (fm) {
        const uint64_t low = (fm & (0ull - fm)) - 1ull;   // bits below the lowest fixed one
        c = ((c & ~low) << 1) | (c & low);
        fm &= fm - 1ull;
    }
    return c | gd.fixed_val;
}

// chunk id of enumerated position `item`
__device__ __forceinline__ uint64_t item_chunk(const GateDesc &gd, uint64_t item)
{
    if (gd.job_type == J_GROUP) {
        uint64_t c = deposit(gd, item >> (gd.pair_bit3 ? 3 : 2));
        return c | ((item & 1ull) ? gd.pair_bit : 0ull) | ((item & 2ull) ? gd.pair_bit2 : 0ull) |
               ((gd.pair_bit3 && (item & 4ull)) ? gd.pair_bit3 : 0ull);
    }
    if (gd.job_type == J_PAIR) {
        uint64_t c = deposit(gd, item >> 1);
        return (item & 1ull) ? (c | gd.pair_bit) : c;
    }
    return deposit(gd, item);
}

// chunk id of position `item` of a job (0 when the position is past the end)
// and whether the job re-encodes it
template <int SRC, bool GATE>
__device__ __forceinline__ bool job_slot(const GateDesc &gd, uint32_t unit_mask, const IOPtrs &io, int cb, uint64_t item,
                                         uint64_t &c)
{
    const bool valid = item < gd.nitems;
    if (SRC == SRC_ARENA && !GATE && io.list) c = valid ? io.list[item] : 0;
    else c = valid ? item_chunk(gd, item) + io.first : 0;
    return valid && !(GATE && gd.check_phase && !diag_touches(gd, unit_mask, c, cb)) &&
           !(GATE && (c & gd.act_mask) != gd.act_val);
}

// validity of a table entry's stream: in the arena, within a staging buffer
__device__ __forceinline__ bool entry_ok(uint64_t entry, uint64_t arena_words)
{
    const uint32_t size = (uint32_t)(entry & 0xFFFFull);
    const uint32_t words = (size + 3u) >> 2;
    return words <= (uint32_t)(kBufWords - 8) && (entry >> 16) + words <= arena_words && size >= 4;
}

// D: a GateDesc, or a fused run's RunRec (the fields kind, q, q2, cm, job_type)
template <class D>
__device__ void apply_gate(const D &gd, const double *m, double *v0, double *v1, uint64_t c0, uint64_t c1,
                           bool a0, bool a1, int cb, int nthreads)
{
    const int tid = threadIdx.x;
    const int ca = 1 << cb;
    // the control test splits into the chunk's index bits (one test per
    // chunk) and the in-chunk bits (one per amplitude)
    const uint64_t cm_hi = gd.cm & ~(uint64_t)(ca - 1);
    const uint32_t cm_lo = (uint32_t)(gd.cm & (uint64_t)(ca - 1));
    const bool hi0 = ((c0 << cb) & cm_hi) == cm_hi, hi1 = ((c1 << cb) & cm_hi) == cm_hi;
    // the matrix in registers (m is an LDS copy that the loops below would
    // otherwise re-read after every store)
    const double u0r = m[0], u0i = m[1], u1r = m[2], u1i = m[3], u2r = m[4], u2i = m[5], u3r = m[6], u3i = m[7];
    if (gd.job_type == J_PAIR) {
        if (!(a0 && a1 && hi0)) return;
        for (int k = tid; k < ca; k += nthreads) {
            if (((uint32_t)k & cm_lo) != cm_lo) continue;
            const int p = vpos(2 * k);
            double ar = v0[p], ai = v0[p + 1], br = v1[p], bi = v1[p + 1];
            if (gd.kind == K_X) {
                v0[p] = br; v0[p + 1] = bi; v1[p] = ar; v1[p + 1] = ai;
            } else {
                double yr, yi, zr, zi;
                lin2(u0r, u0i, u1r, u1i, ar, ai, br, bi, yr, yi);
                lin2(u2r, u2i, u3r, u3i, ar, ai, br, bi, zr, zi);
                v0[p] = yr; v0[p + 1] = yi; v1[p] = zr; v1[p + 1] = zi;
            }
        }
        return;
    }
    const bool pairwise = gd.kind == K_U1 || gd.kind == K_X;
    const int units = pairwise ? ca / 2 : ca;
    for (int s = 0; s < 2; ++s) {
        if (!(s ? (a1 && hi1) : (a0 && hi0))) continue;
        double *v = s ? v1 : v0;
        for (int u = tid; u < units; u += nthreads) {
            if (pairwise) {
                const int q = gd.q;
                const int k0 = ((u >> q) << (q + 1)) | (u & ((1 << q) - 1));
                const int k1 = k0 | (1 << q);
                if (((uint32_t)k0 & cm_lo) != cm_lo) continue;
                const int p0 = vpos(2 * k0), p1 = vpos(2 * k1);
                double ar = v[p0], ai = v[p0 + 1], br = v[p1], bi = v[p1 + 1];
                if (gd.kind == K_X) {
                    v[p0] = br; v[p0 + 1] = bi; v[p1] = ar; v[p1 + 1] = ai;
                } else {
                    double yr, yi, zr, zi;
                    lin2(u0r, u0i, u1r, u1i, ar, ai, br, bi, yr, yi);
                    lin2(u2r, u2i, u3r, u3i, ar, ai, br, bi, zr, zi);
                    v[p0] = yr; v[p0 + 1] = yi; v[p1] = zr; v[p1 + 1] = zi;
                }
            } else {
                if (((uint32_t)u & cm_lo) != cm_lo) continue;
                const int p = vpos(2 * u);
                if (gd.kind == K_MCZ) {
                    v[p] = -v[p];
                    v[p + 1] = -v[p + 1];
                } else {
                    const uint64_t i = ((s ? c1 : c0) << cb) | (uint64_t)u;
                    int idx = (int)((i >> gd.q) & 1ull);
                    if (gd.kind == K_DIAG2) idx += 2 * (int)((i >> gd.q2) & 1ull);
                    double yr, yi, pr, pi;
                    phase_of(m, idx, pr, pi);
                    dmul(pr, pi, v[p], v[p + 1], yr, yi);
                    v[p] = yr; v[p + 1] = yi;
                }
            }
        }
    }
}

// A fused run's gate as the run loop reads it, copied to LDS once per launch:
// the kernel writes global memory, so reads of the run's records there inside
// the job loop would be vector loads, each waited for on its own.
static_assert(kMaxRun <= 64, "a run's touch masks are wavefront ballots: one lane per gate");
struct RunRec {
    uint64_t cm;                     // control mask over amplitude-index bits
    uint64_t fixed_mask, fixed_val;  // chunk-index bits held fixed by the gate's enumeration
    int32_t kind, q, q2, job_type;
    int32_t check_phase;             // diagonal: chunks whose reachable phases are all 1 are not touched
    uint32_t unit;                   // bit i: phase i is 1
};

__device__ __forceinline__ RunRec run_rec(const GateDesc &d)
{
    RunRec r;
    r.cm = d.cm;
    r.fixed_mask = d.fixed_mask;
    r.fixed_val = d.fixed_val;
    r.kind = d.kind;
    r.q = d.q;
    r.q2 = d.q2;
    r.job_type = d.job_type;
    r.check_phase = d.check_phase;
    r.unit = 0;
    for (int i = 0; i < 4; ++i) r.unit |= unit_phase(d.m[2 * i], d.m[2 * i + 1]) ? (1u << i) : 0u;
    return r;
}

// wave-uniform values read from LDS: held in scalar registers, so that tests
// and branches on them are scalar instructions instead of per-lane masks
__device__ __forceinline__ uint32_t uni32(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }
__device__ __forceinline__ int32_t uni32(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uni64(uint64_t v)
{
    return ((uint64_t)uni32((uint32_t)(v >> 32)) << 32) | uni32((uint32_t)v);
}

__device__ __forceinline__ RunRec uniform_rec(const RunRec &r)
{
    RunRec u;
    u.cm = uni64(r.cm);
    u.fixed_mask = uni64(r.fixed_mask);
    u.fixed_val = uni64(r.fixed_val);
    u.kind = uni32(r.kind);
    u.q = uni32(r.q);
    u.q2 = uni32(r.q2);
    u.job_type = uni32(r.job_type);
    u.check_phase = uni32(r.check_phase);
    u.unit = uni32(r.unit);
    return u;
}

// whether gate rg of a fused run re-encodes chunk c: the chunk is in its
// enumeration (controls on chunk-index qubits, a diagonal's fixed half) and,
// for a diagonal gate, some phase reachable in the chunk is not 1
__device__ __forceinline__ bool run_touches(const RunRec &rg, uint64_t c, int cb)
{
    if ((c & rg.fixed_mask) != rg.fixed_val) return false;
    if (!rg.check_phase) return true;
    return diag_touches(rg, rg.unit, c, cb);
}

// A single-chunk gate that each thread can apply to its own V values: diagonal
// phases, multi-controlled Z, and U1 / X whose target pairs lie inside a
// thread's V/2 amplitudes (2^(q+1) <= V/2).  Same arithmetic as apply_gate.
template <int V, class D>
__device__ __forceinline__ bool gate_in_registers(const D &gd)
{
    if (gd.job_type != J_SINGLE || (V & 1)) return false;
    if (gd.kind == K_DIAG1 || gd.kind == K_DIAG2 || gd.kind == K_MCZ) return true;
    return (gd.kind == K_U1 || gd.kind == K_X) && (2 << gd.q) <= V / 2;
}

// A thread holds amplitudes base .. base + V/2 - 1 with base a multiple of
// V/2: an amplitude index splits into the thread's fixed high bits and the
// low bits a (a compile-time loop index).  Control tests and phase indices
// are split the same way, so the per-amplitude part is uniform over the wave.
template <int V>
struct RegSplit {
    static constexpr int A = V / 2;                                // amplitudes per thread
    static constexpr int LB = A >= 8 ? 3 : A >= 4 ? 2 : A >= 2 ? 1 : 0;   // log2(A)
    bool mine;       // my high bits satisfy the high controls
    uint32_t cm_lo;  // controls among the low bits
    template <class D>
    __device__ __forceinline__ RegSplit(const D &gd, uint64_t base)
    {
        const uint64_t hi_mask = ~(uint64_t)(A - 1);
        mine = (base & gd.cm & hi_mask) == (gd.cm & hi_mask);
        cm_lo = (uint32_t)(gd.cm & (uint64_t)(A - 1));
    }
};

template <int V, int Q, class D>
__device__ __forceinline__ void pairs_in_registers(const D &gd, const double *m, double (&x)[V],
                                                   const RegSplit<V> &sp)
{
#pragma unroll
    for (int a = 0; a < V / 2; ++a) {
        if (a & (1 << Q)) continue;
        const int a1 = a | (1 << Q);
        if (((uint32_t)a & sp.cm_lo) != sp.cm_lo) continue;
        const double ar = x[2 * a], ai = x[2 * a + 1], br = x[2 * a1], bi = x[2 * a1 + 1];
        if (gd.kind == K_X) {
            x[2 * a] = br; x[2 * a + 1] = bi; x[2 * a1] = ar; x[2 * a1 + 1] = ai;
        } else {
            double yr, yi, zr, zi;
            lin2(m[0], m[1], m[2], m[3], ar, ai, br, bi, yr, yi);
            lin2(m[4], m[5], m[6], m[7], ar, ai, br, bi, zr, zi);
            x[2 * a] = yr; x[2 * a + 1] = yi; x[2 * a1] = zr; x[2 * a1 + 1] = zi;
        }
    }
}

// x: my V values (amplitudes base .. base + V/2 - 1 of the state)
template <int V, class D>
__device__ __forceinline__ void apply_gate_registers(const D &gd, const double *m, double (&x)[V], uint64_t base)
{
    const RegSplit<V> sp(gd, base);
    if (!sp.mine) return;
    constexpr int LB = RegSplit<V>::LB;
    if (gd.kind == K_U1 || gd.kind == K_X) {
        if (gd.q == 0) pairs_in_registers<V, 0>(gd, m, x, sp);
        else if (gd.q == 1 && V >= 8) pairs_in_registers<V, (V >= 8 ? 1 : 0)>(gd, m, x, sp);
        else if (gd.q == 2 && V >= 16) pairs_in_registers<V, (V >= 16 ? 2 : 0)>(gd, m, x, sp);
        return;
    }
    if (gd.kind == K_MCZ) {
#pragma unroll
        for (int a = 0; a < V / 2; ++a) {
            if (((uint32_t)a & sp.cm_lo) != sp.cm_lo) continue;
            x[2 * a] = -x[2 * a];
            x[2 * a + 1] = -x[2 * a + 1];
        }
        return;
    }
    // diagonal: phase index bit 0 from qubit q, bit 1 from qubit q2 (DIAG2)
    const int q = gd.q, q2 = gd.kind == K_DIAG2 ? gd.q2 : -1;
    const bool q_lo = q < LB, q2_lo = q2 >= 0 && q2 < LB;
    uint32_t ihi = 0;
    if (!q_lo) ihi |= (uint32_t)(base >> q) & 1u;
    if (q2 >= 0 && !q2_lo) ihi |= ((uint32_t)(base >> q2) & 1u) << 1;
    if (!q_lo && !q2_lo) {
        // one phase for all my amplitudes
        double pr, pi;
        phase_of(m, (int)ihi, pr, pi);
#pragma unroll
        for (int a = 0; a < V / 2; ++a) {
            if (((uint32_t)a & sp.cm_lo) != sp.cm_lo) continue;
            double yr, yi;
            dmul(pr, pi, x[2 * a], x[2 * a + 1], yr, yi);
            x[2 * a] = yr; x[2 * a + 1] = yi;
        }
        return;
    }
#pragma unroll
    for (int a = 0; a < V / 2; ++a) {
        if (((uint32_t)a & sp.cm_lo) != sp.cm_lo) continue;
        const uint32_t idx = ihi | (q_lo ? ((uint32_t)a >> q) & 1u : 0u) | (q2_lo ? (((uint32_t)a >> q2) & 1u) << 1 : 0u);
        double yr, yi, pr, pi;
        phase_of(m, (int)idx, pr, pi);
        dmul(pr, pi, x[2 * a], x[2 * a + 1], yr, yi);
        x[2 * a] = yr; x[2 * a + 1] = yi;
    }
}

// A diagonal gate without controls: in a fused run such gates take a loop of
// their own (see the job kernel), one phase per thread when its qubits lie
// above the thread's low index bits, else one per amplitude.
template <int V>
__device__ __forceinline__ bool thread_phase_diag(const RunRec &rg)
{
    return (V & 1) == 0 && V >= 2 && rg.job_type == J_SINGLE && (rg.kind == K_DIAG1 || rg.kind == K_DIAG2) &&
           rg.cm == 0;
}

// An uncontrolled U1 / X on an in-chunk qubit whose pairs span threads: in a
// fused run consecutive such gates are applied in LDS one after another
// (see the job kernel).
template <int V>
__device__ __forceinline__ bool lds_pair_gate(const RunRec &rg)
{
    return rg.job_type == J_SINGLE && (rg.kind == K_U1 || rg.kind == K_X) && rg.cm == 0 && !gate_in_registers<V>(rg);
}

// One such gate on the slots' chunks in LDS (apply_gate's pair update), each
// value tested for a subnormal result and truncated as it is written; a slot
// whose chunk the gate does not touch (t0 / t1 false) is left alone.
__device__ __forceinline__ void lds_pairs_truncated(const RunRec &rg, const double *m, double *v0, double *v1, bool t0,
                                                    bool t1, int cb, int nthreads, uint64_t m64, bool &seen)
{
    const int tid = threadIdx.x;
    const int units = (1 << cb) / 2;
    const int q = rg.q;
    const double u0r = m[0], u0i = m[1], u1r = m[2], u1i = m[3], u2r = m[4], u2i = m[5], u3r = m[6], u3i = m[7];
    for (int s = 0; s < 2; ++s) {
        if (!(s ? t1 : t0)) continue;
        double *v = s ? v1 : v0;
        for (int u = tid; u < units; u += nthreads) {
            const int k0 = ((u >> q) << (q + 1)) | (u & ((1 << q) - 1));
            const int k1 = k0 | (1 << q);
            const int p0 = vpos(2 * k0), p1 = vpos(2 * k1);
            double ar = v[p0], ai = v[p0 + 1], br = v[p1], bi = v[p1 + 1];
            if (rg.kind == K_X) {
                const double tr = ar, ti = ai;
                ar = br; ai = bi; br = tr; bi = ti;
            } else {
                double yr, yi, zr, zi;
                lin2(u0r, u0i, u1r, u1i, ar, ai, br, bi, yr, yi);
                lin2(u2r, u2i, u3r, u3i, ar, ai, br, bi, zr, zi);
                ar = yr; ai = yi; br = zr; bi = zi;
            }
            seen |= is_subnormal(ar);
            seen |= is_subnormal(ai);
            seen |= is_subnormal(br);
            seen |= is_subnormal(bi);
            v[p0] = u2d(d2u(ar) & m64);
            v[p0 + 1] = u2d(d2u(ai) & m64);
            v[p1] = u2d(d2u(br) & m64);
            v[p1 + 1] = u2d(d2u(bi) & m64);
        }
    }
}

// ---------------------------------------------------------------------------
// the job kernel
// ---------------------------------------------------------------------------
// Two-wavefront groups run three workgroups per CU (three waves per SIMD):
// the phases of a job wait on HBM, the arena atomic and barriers, and a third
// workgroup keeps the SIMDs busy meanwhile; that caps a thread at 168 VGPRs.
// block cache (Sec. 3.4): chunk-index bits whose values the gate reads
// (controls, and diagonal targets above the chunk); two jobs whose chunks
// agree on them get the same operation
__device__ __forceinline__ uint64_t op_mask(const GateDesc &gd, int cb)
{
    uint64_t m = gd.cm >> cb;
    if (gd.q >= cb) m |= 1ull << (gd.q - cb);
    if (gd.kind == K_DIAG2 && gd.q2 >= cb) m |= 1ull << (gd.q2 - cb);
    return m;
}

// LIST 0: every job of the launch.  LIST 3: a fused run of in-chunk gates
// (io.run), each followed by the truncation its re-encoding would apply, with
// one decode before and one encode after.  With the block cache, LIST 1 runs the
// leader jobs and leaves the gate open; LIST 2 computes the followers that the
// copy kernel did not copy (their bytes differ from their leader's) and closes
// the gate over the leaders' launch, the copy kernel and itself.
template <int V, int WPG, int SRC, int DST, bool GATE, int LIST = 0, bool ENT = false>
__global__ __launch_bounds__(128 * WPG, WPG == 2 ? 3 : 1) void job_kernel(GateDesc gd, DevPtrs P, IOPtrs io)
{
    constexpr int G = 64 * WPG;   // threads per chunk slot
    constexpr int WGS = 2 * G;    // threads per workgroup
    __shared__ __align__(16) uint32_t buf[2][kBufWords];
    __shared__ uint32_t sh[256];
    __shared__ uint64_t sh_off[2];
    __shared__ int sh_ok[2];
    __shared__ int sh_src_ok[2];
    __shared__ uint64_t sh_acc[8];
    __shared__ double sh_mom[WGS / 64][4];
    __shared__ double sh_cs[DST == DST_CSTATS ? WGS / 64 : 1][9];
    // the gate's parameters: read in the gate phase from LDS, so that the job
    // loop does not hold them in scalar registers
    __shared__ double sh_m[8];
    __shared__ double sh_rm[LIST == 3 ? kMaxRun : 1][8];   // fused run: the gates' matrices
    __shared__ uint32_t sh_rsub[2][WGS / 64];              // fused run: subnormal flags, alternating per truncation
    __shared__ RunRec sh_rr[LIST == 3 ? kMaxRun : 1];      // fused run: the gates' records
    // entropy stage, per slot: decode tables while decoding, encode tables and lane records while encoding
    __shared__ __align__(16) uint32_t sh_ent[ENT ? 2 : 1][ENT ? kEntSlotWords : 1];

    DevState *ds = P.ds;
    if (DST == DST_ARENA && ds->stop) return;

    const int tid = threadIdx.x, s = tid / G, lt = tid % G;
    if (GATE && tid < 8) sh_m[tid] = gd.m[tid];   // first read after the first job's fetch barrier
    uint64_t fastm = 0;   // fused run: bit g set when gate g is an uncontrolled diagonal gate (thread_phase_diag)
    uint64_t ldsm = 0;    // fused run: bit g set when gate g is an LDS pair gate (lds_pair_gate)
    if (LIST == 3) {
        for (int i = tid; i < 8 * io.nrun; i += WGS) sh_rm[i >> 3][i & 7] = io.run[i >> 3].m[i & 7];
        for (int g = tid; g < io.nrun; g += WGS) sh_rr[g] = run_rec(io.run[g]);
        lds_barrier();   // the records are read before the first job's fetch barrier
        const int ln = tid & 63;
        fastm = __ballot(ln < io.nrun && thread_phase_diag<V>(sh_rr[ln < io.nrun ? ln : 0]));
        ldsm = __ballot(ln < io.nrun && lds_pair_gate<V>(sh_rr[ln < io.nrun ? ln : 0]));
    }
    uint32_t unit_mask = 0;                        // phases equal to 1 (diagonal gates)
    if (GATE)
        for (int i = 0; i < 4; ++i) unit_mask |= unit_phase(gd.m[2 * i], gd.m[2 * i + 1]) ? (1u << i) : 0u;
    const int C = P.C;
    uint32_t *b = buf[s];
    double *vals = reinterpret_cast<double *>(b);
    const int first = lt * V;
    // LDS slots of the scans (per call site)
    uint32_t *slA = sh, *slB = sh + 16, *slC = sh + 32, *slE = sh + 48, *slF = sh + 176, *slS = sh + 192,
             *slD = sh + 224;
    uint32_t *ent = sh_ent[ENT ? s : 0];
    const bool ent_on = ENT && gd.entropy != 0;
    const int glevel = (DST == DST_ARENA || DST == DST_SLOTS) && gd.fixed_level < 0 && !gd.per_block ? ds->level : 0;
    const uint64_t ds_nstripes = DST == DST_ARENA ? ds->nstripes : 1;
    const uint64_t ds_base = DST == DST_ARENA ? ds->base : 0;           // fixed while a gate runs
    const uint64_t ds_ssize = DST == DST_ARENA ? ds->stripe_size : 0;

    // per-slot totals (size change, re-encoded chunks, bytes read, bytes
    // written) live in LDS: only thread 0 of a slot updates them
    if (DST == DST_ARENA && lt == 0)
        for (int k = 0; k < 4; ++k) sh_acc[4 * s + k] = 0;
    double acc_wd = 0.0, acc_lost = 0.0;   // per-block fidelity ledger terms
    double mom_re = 0.0, mom_im = 0.0, mom_n2 = 0.0;

    const uint64_t jstop = job_stop(gd);
    __shared__ uint32_t sh_role[(LIST == 1 || LIST == 2) ? 256 : 1];
    uint32_t kjob = 0;   // iterations of this workgroup's job loop
    for (uint64_t job = job_begin(gd) + blockIdx.x; job < jstop; job += gridDim.x, ++kjob) {
        uint32_t rjob = 0;
        if (LIST == 1 || LIST == 2) {
            if ((kjob & 255u) == 0u) {   // the roles of this workgroup's next 256 jobs, in one batch
                lds_barrier();
                const uint64_t jj = job + (uint64_t)tid * gridDim.x;
                if (tid < 256) sh_role[tid] = jj < jstop ? io.role[jj - job_begin(gd)] : 0u;
                lds_barrier();
            }
            rjob = sh_role[kjob & 255u];
            if (LIST == 1 ? rjob != 0u : (rjob == 0u || rjob == kRoleDone)) continue;   // (uniform over the workgroup)
        }
        const uint64_t item0 = 2 * job, item1 = 2 * job + 1;
        const bool valid0 = item0 < gd.nitems, valid1 = item1 < gd.nitems;
        uint64_t cc0 = 0, cc1 = 0;
        bool act0 = job_slot<SRC, GATE>(gd, unit_mask, io, P.cb, item0, cc0);
        bool act1 = job_slot<SRC, GATE>(gd, unit_mask, io, P.cb, item1, cc1);
        uint64_t tm0 = 0, tm1 = 0;   // fused run: bit g set when gate g touches the slot's chunk
        if (LIST == 3) {
            // a fused run enumerates every chunk; it re-encodes those some gate
            // touches.  Lane g of every wavefront tests gate g (at most 64 gates
            // per run), and the ballots give each wavefront both masks.
            const int ln = tid & 63;
            const bool in_run = ln < io.nrun;
            tm0 = __ballot(in_run && run_touches(sh_rr[in_run ? ln : 0], cc0, P.cb));
            tm1 = __ballot(in_run && run_touches(sh_rr[in_run ? ln : 0], cc1, P.cb));
            act0 = act0 && tm0 != 0;
            act1 = act1 && tm1 != 0;
        }
        const uint64_t item = s ? item1 : item0;
        const uint64_t c = s ? cc1 : cc0;
        const bool valid = s ? valid1 : valid0;
        const bool act = s ? act1 : act0;

        // 1-3. fetch, decode and (fused runs) the run's gates; a fused run
        // takes a second attempt when its first one met a subnormal value
        uint64_t old_entry = 0;
        bool ok_src = true, use0 = false, use1 = false, use = false;
        uint32_t my_hdr = 0;
        bool verified = false;   // a fused run's truncation steps found no subnormal value
        for (bool careful = false;; careful = true) {
            // 1. fetch
            old_entry = 0;
            ok_src = true;
            if (SRC == SRC_ARENA) {
                if (valid) old_entry = P.table[c];
                const uint32_t size = (uint32_t)(old_entry & 0xFFFFull);
                const uint64_t off = old_entry >> 16;
                const uint32_t words = (size + 3u) >> 2;
                ok_src = entry_ok(old_entry, P.arena_words);
                if (act && ok_src) {
                    if ((off & 3ull) == 0) stage_units<G>(b, P.arena + off, words, lt);
                    else stage_words<G>(b, P.arena + off, words, lt);
                }
                if ((act || (GATE && gd.sweep && valid)) && !ok_src && lt == 0 && ds) atomicExch(&ds->corrupt, 1);
            } else if (SRC == SRC_SLOTS) {
                const uint32_t size = valid ? io.sizes_in[item] : 0u;
                const uint32_t words = (size + 3u) >> 2;
                ok_src = words <= (uint32_t)(kBufWords - 8) && words <= io.slot_words && size >= 4;
                if (act && ok_src) stage_words<G>(b, io.slots_in + item * io.slot_words, words, lt);
            } else {  // SRC_RAW
                if (act)
                    for (int w = lt; w < C; w += G) vals[vpos(w)] = io.raw_in[item * (uint64_t)C + w];
            }
            if (lt == 0) sh_src_ok[s] = ok_src ? 1 : 0;
            lds_barrier();
            // (slot streams of Solution B, header mode 3, are decoded by their own kernel)
            use0 = act0 && sh_src_ok[0] != 0 && (SRC != SRC_SLOTS || (buf[0][0] & 3u) != 3u);
            use1 = act1 && sh_src_ok[1] != 0 && (SRC != SRC_SLOTS || (buf[1][0] & 3u) != 3u);
            use = s ? use1 : use0;

            // 2. decode
            my_hdr = 0;
            if (SRC != SRC_RAW) {
                const uint32_t hdr0 = use0 ? buf[0][0] : (uint32_t)M_CONST2;
                const uint32_t hdr1 = use1 ? buf[1][0] : (uint32_t)M_CONST2;
                my_hdr = s ? hdr1 : hdr0;
                const bool any_sparse = (hdr0 & 3u) == M_SPARSE || (hdr1 & 3u) == M_SPARSE;
                const bool any_ent = ENT && ((hdr0 | hdr1) & kHdrEnt) != 0;
                uint32_t th[V], tl[V];
                decode_group<V, WPG, ENT>(b, s ? hdr1 : hdr0, use, any_sparse, C, lt, slA, slB, slC, th, tl, any_ent,
                                          reinterpret_cast<uint8_t *>(ent));
                lds_barrier();
                double x[V];
#pragma unroll
                for (int k = 0; k < V; ++k) x[k] = u2d(((uint64_t)th[k] << 32) | tl[k]);
                // Solution D streams: the values, decoded in stored order, go to their
                // interleaved positions through LDS (uniform branch over the workgroup)
                const bool rsh0 = use0 && (hdr0 & kHdrRsh) != 0, rsh1 = use1 && (hdr1 & kHdrRsh) != 0;
                if (rsh0 || rsh1) {
                    const bool mine = s ? rsh1 : rsh0;
                    store_interleaved<V>(vals, first, C, mine, x);
                    lds_barrier();
#pragma unroll
                    for (int k = 0; k < V; ++k) x[k] = vals[vpos(first + k)];
                }
                if (LIST == 3) {
                    // 3r. the run: each gate (in registers or through LDS), then the
                    // truncation re-encoding would apply, none when the chunk holds a
                    // subnormal value, so that the one encode below equals the last
                    // of the gate-by-gate encodes.  The first attempt truncates after
                    // every gate and notes whether a touched value came out
                    // subnormal; if one did in either slot, both chunks are fetched
                    // and run again, this time deciding over the whole chunk after
                    // each gate (a barrier per gate).
                    const uint64_t base = (c << P.cb) | (uint64_t)(first / 2);
                    const uint32_t mh = sig_mask_hi(sig_bits(glevel));
                    bool seen = false;   // a touched value of mine came out subnormal
                    int ntr = 0;
                    // (a wavefront lies in one slot: its slot's mask and chunk state are wave-uniform)
                    const uint64_t tm_w = uni64(s ? tm1 : tm0);
                    const bool use_w = uni32((uint32_t)(s ? use1 : use0)) != 0;
                    for (int g = 0; g < io.nrun;) {
                        if (!careful && glevel > 0 && ((fastm >> g) & 1ull) != 0) {
                            // consecutive uncontrolled diagonal gates: the ones that
                            // touch my chunk, each with the update, the subnormal test
                            // and the truncation in one pass over my values (a loop of
                            // their own, without branches on the gate kind)
                            const uint64_t rest = ~(fastm >> g);
                            const int e = rest != 0 ? g + __builtin_ctzll(rest) : 64;   // end of the segment
                            const uint64_t seg = e - g >= 64 ? ~0ull : ((1ull << (e - g)) - 1ull);
                            uint64_t todo = use_w ? (tm_w >> g) & seg : 0ull;
                            const uint64_t m64 = (uint64_t)mh << 32;   // the truncation as one mask
                            while (todo != 0) {
                                const int k = g + __builtin_ctzll(todo);
                                todo &= todo - 1ull;
                                const RunRec rk = uniform_rec(sh_rr[k]);
                                // phase index bits from my high index bits (the low ones of
                                // base are 0), then per amplitude those of a low qubit
                                uint32_t ihi = (uint32_t)(base >> rk.q) & 1u;
                                if (rk.kind == K_DIAG2) ihi |= ((uint32_t)(base >> rk.q2) & 1u) << 1;
                                constexpr int LB = RegSplit<V>::LB;
                                const int ql = rk.q < LB ? rk.q : LB;
                                const int q2l = (rk.kind == K_DIAG2 && rk.q2 < LB) ? rk.q2 : LB;
                                if (ql == LB && q2l == LB) {
                                    double pr, pi;
                                    phase_of(sh_rm[k], (int)ihi, pr, pi);
#pragma unroll
                                    for (int a = 0; a < V / 2; ++a) {
                                        double yr, yi;
                                        dmul(pr, pi, x[2 * a], x[2 * a + 1], yr, yi);
                                        seen |= is_subnormal(yr);
                                        seen |= is_subnormal(yi);
                                        x[2 * a] = u2d(d2u(yr) & m64);
                                        x[2 * a + 1] = u2d(d2u(yi) & m64);
                                    }
                                } else {
#pragma unroll
                                    for (int a = 0; a < V / 2; ++a) {
                                        const uint32_t idx = ihi | (((uint32_t)a >> ql) & 1u) | ((((uint32_t)a >> q2l) & 1u) << 1);
                                        double pr, pi, yr, yi;
                                        phase_of(sh_rm[k], (int)idx, pr, pi);
                                        dmul(pr, pi, x[2 * a], x[2 * a + 1], yr, yi);
                                        seen |= is_subnormal(yr);
                                        seen |= is_subnormal(yi);
                                        x[2 * a] = u2d(d2u(yr) & m64);
                                        x[2 * a + 1] = u2d(d2u(yi) & m64);
                                    }
                                }
                            }
                            g = e;
                            continue;
                        }
                        if (!careful && glevel > 0 && ((ldsm >> g) & 1ull) != 0 && ((ldsm >> g) & 2ull) != 0) {
                            // two or more consecutive LDS pair gates: my values go to LDS
                            // once, each gate updates, tests and truncates the pairs of
                            // the chunks it touches, and they come back at the end
                            const uint64_t rest = ~(ldsm >> g);
                            const int e = rest != 0 ? g + __builtin_ctzll(rest) : 64;   // end of the segment
                            const uint64_t m64 = (uint64_t)mh << 32;
#pragma unroll
                            for (int k = 0; k < V; ++k) vals[vpos(first + k)] = x[k];
                            for (; g < e; ++g) {
                                lds_barrier();
                                const RunRec rj = uniform_rec(sh_rr[g]);
                                lds_pairs_truncated(rj, sh_rm[g], reinterpret_cast<double *>(buf[0]),
                                                    reinterpret_cast<double *>(buf[1]),
                                                    use0 && ((tm0 >> g) & 1ull) != 0, use1 && ((tm1 >> g) & 1ull) != 0,
                                                    P.cb, WGS, m64, seen);
                            }
                            lds_barrier();
#pragma unroll
                            for (int k = 0; k < V; ++k) x[k] = vals[vpos(first + k)];
                            continue;
                        }
                        const RunRec rg = uniform_rec(sh_rr[g]);
                        // a chunk the gate does not touch skips it and its truncation,
                        // as it would keep its stream gate by gate
                        const bool tg0 = use0 && ((tm0 >> g) & 1ull) != 0, tg1 = use1 && ((tm1 >> g) & 1ull) != 0;
                        const bool tg = s ? tg1 : tg0;
                        if (gate_in_registers<V>(rg)) {
                            if (tg) apply_gate_registers<V>(rg, sh_rm[g], x, base);
                        } else {
#pragma unroll
                            for (int k = 0; k < V; ++k) vals[vpos(first + k)] = x[k];
                            lds_barrier();
                            apply_gate(rg, sh_rm[g], reinterpret_cast<double *>(buf[0]),
                                       reinterpret_cast<double *>(buf[1]), cc0, cc1, tg0, tg1, P.cb, WGS);
                            lds_barrier();
#pragma unroll
                            for (int k = 0; k < V; ++k) x[k] = vals[vpos(first + k)];
                        }
                        if (glevel > 0 && (tg0 || tg1)) {
                            bool sub = false;
#pragma unroll
                            for (int k = 0; k < V; ++k) sub = sub || is_subnormal(x[k]);
                            uint32_t gs = 0;
                            if (careful) {
                                const bool wsub = __any(tg && sub);
                                if ((tid & 63) == 0) sh_rsub[ntr & 1][tid >> 6] = wsub ? 1u : 0u;
                                lds_barrier();
#pragma unroll
                                for (int i = 0; i < WPG; ++i) gs |= sh_rsub[ntr & 1][s * WPG + i];
                                ++ntr;   // flags alternate per truncation step: a barrier separates reuses
                            } else {
                                seen = seen || (tg && sub);
                            }
                            if (gs == 0 && tg) {
#pragma unroll
                                for (int k = 0; k < V; ++k) x[k] = u2d((uint64_t)((uint32_t)(d2u(x[k]) >> 32) & mh) << 32);
                            }
                        }
                        ++g;
                    }
                    if (!careful && glevel > 0) {
                        // (sh_rsub is next written after the fetch barrier of the
                        // second attempt or of a later job)
                        const bool wsub = __any(seen);
                        if ((tid & 63) == 0) sh_rsub[0][tid >> 6] = wsub ? 1u : 0u;
                        lds_barrier();
                        uint32_t any = 0;
#pragma unroll
                        for (int i = 0; i < WGS / 64; ++i) any |= sh_rsub[0][i];
                        if (any != 0) continue;   // (uniform over the workgroup)
                        verified = true;
                    }
                } else if (GATE && gate_in_registers<V>(gd) && use) {
                    // 3a. a gate each thread applies to its own values (no LDS pass)
                    apply_gate_registers<V>(gd, sh_m, x, (c << P.cb) | (uint64_t)(first / 2));
                }
#pragma unroll
                for (int k = 0; k < V; ++k) vals[vpos(first + k)] = x[k];
                lds_barrier();
            }
            break;
        }

        // 3. gate (pairs across threads or slots, in LDS)
        if (GATE && LIST != 3 && !gate_in_registers<V>(gd)) {
            apply_gate(gd, sh_m, reinterpret_cast<double *>(buf[0]), reinterpret_cast<double *>(buf[1]), cc0, cc1, use0,
                       use1, P.cb, WGS);
            lds_barrier();
        }

        // 4. sink
        if (DST == DST_RAW) {
            if (use)
                for (int w = lt; w < C; w += G) io.raw_out[item * (uint64_t)C + w] = vals[vpos(w)];
        } else if (DST == DST_MOMENTS) {
            if (use) {
#pragma unroll
                for (int k = 0; k < V; k += 2) {
                    double re = vals[vpos(first + k)], im = (k + 1 < V) ? vals[vpos(first + k + 1)] : 0.0;
                    mom_re += re;
                    mom_im += im;
                    mom_n2 += re * re + im * im;
                }
                if (V == 1) {  // one value per thread: odd threads hold the imaginary parts
                    double v = vals[vpos(first)];
                    mom_re -= (lt & 1) ? v : 0.0;
                    mom_im += (lt & 1) ? v : 0.0;
                }
            }
        } else if (DST == DST_CSTATS) {
            // 4a. statistics of the stored values of the chunk
            double n2 = 0.0;
            uint32_t nz = 0, esum = 0, eq8 = 0, eq16 = 0, eq24 = 0, sgn = 0;
            int emax = -1, emin = 4096;
            uint64_t prev = lt ? d2u(vals[vpos(first - 1)]) : 0ull;
#pragma unroll
            for (int k = 0; k < V; ++k) {
                const double x = vals[vpos(first + k)];
                const uint64_t u = d2u(x);
                n2 += x * x;
                const bool isnz = x != 0.0;
                const int e = (int)((u >> 52) & 0x7FFull);
                nz += isnz ? 1u : 0u;
                esum += isnz ? (uint32_t)e : 0u;
                emax = isnz ? max(emax, e) : emax;
                emin = isnz ? min(emin, e) : emin;
                eq8 += (u >> 56) == (prev >> 56) ? 1u : 0u;
                eq16 += (u >> 48) == (prev >> 48) ? 1u : 0u;
                eq24 += (u >> 40) == (prev >> 40) ? 1u : 0u;
                sgn += (u >> 63) != (prev >> 63) ? 1u : 0u;
                prev = u;
            }
            for (int d = 32; d >= 1; d >>= 1) {
                n2 += __shfl_down(n2, d, 64);
                nz += __shfl_down(nz, d, 64);
                esum += __shfl_down(esum, d, 64);
                emax = max(emax, __shfl_down(emax, d, 64));
                emin = min(emin, __shfl_down(emin, d, 64));
                eq8 += __shfl_down(eq8, d, 64);
                eq16 += __shfl_down(eq16, d, 64);
                eq24 += __shfl_down(eq24, d, 64);
                sgn += __shfl_down(sgn, d, 64);
            }
            double *red = sh_cs[tid >> 6];
            if ((tid & 63) == 0) {
                red[0] = n2; red[1] = nz; red[2] = esum; red[3] = emax; red[4] = emin;
                red[5] = eq8; red[6] = eq16; red[7] = eq24; red[8] = sgn;
            }
            lds_barrier();
            if (lt == 0 && use) {
                double r[9];
                for (int j = 0; j < 9; ++j) r[j] = sh_cs[s * WPG][j];
                for (int w = 1; w < WPG; ++w) {
                    const double *o = sh_cs[s * WPG + w];
                    r[0] += o[0]; r[1] += o[1]; r[2] += o[2];
                    r[3] = fmax(r[3], o[3]); r[4] = fmin(r[4], o[4]);
                    r[5] += o[5]; r[6] += o[6]; r[7] += o[7]; r[8] += o[8];
                }
                double *out = io.cstats + (c - io.first) * kChunkStats;
                for (int j = 0; j < 9; ++j) out[j] = r[j];
                out[CS_CONST2] = (my_hdr & 3u) == (uint32_t)M_CONST2 ? 1.0 : 0.0;
                out[CS_BYTES] = (double)(((old_entry & 0xFFFFull) + 3ull) & ~3ull);
                out[11] = 0.0;
            }
        } else if (DST == DST_LSIZES) {
            // 4b. padded size of the chunk re-encoded at every level
            uint32_t xh[V], xl[V];
            bool sub = false;
            const bool rsh = gd.reshuffle != 0;   // values in Solution D's stored order
            load_stored<V>(vals, first, C, rsh, xh, xl, sub);
            const uint32_t xprev_hi =
                lt ? (uint32_t)(d2u(vals[vpos(rsh ? rsh_pos(first - 1, C) : first - 1)]) >> 32) : 0u;
            const uint64_t x0 = d2u(vals[0]), x1 = d2u(vals[1]);
            const bool wsub = __any(use && sub);
            if ((tid & 63) == 0) slS[tid >> 6] = wsub ? 1u : 0u;
            lds_barrier();
            uint32_t gs = 0;
#pragma unroll
            for (int i = 0; i < WPG; ++i) gs |= slS[s * WPG + i];
            for (int lev = 0; lev < kLevels; ++lev) {
                EncPlan<V> e;
                encode_plan<V, WPG, ENT>(xh, xl, xprev_hi, x0, x1, lev, gs != 0, C, lt, slE, slF, e, ent_on, b, ent,
                                         slD, rsh);
                if (lt == 0 && use)
                    atomicAdd((unsigned long long *)&io.lsizes[(c >> gd.block_shift) * kLevels + lev],
                              (unsigned long long)((e.size + 3u) & ~3u));
                lds_barrier();
            }
        } else {
            // encode at the chunk's level
            uint32_t xh[V], xl[V];
            bool sub = false;
            const bool rsh = gd.reshuffle != 0;   // values in Solution D's stored order
            load_stored<V>(vals, first, C, rsh, xh, xl, sub);
            const uint32_t xprev_hi =
                lt ? (uint32_t)(d2u(vals[vpos(rsh ? rsh_pos(first - 1, C) : first - 1)]) >> 32) : 0u;
            const uint64_t x0 = d2u(vals[0]), x1 = d2u(vals[1]);
            int lev_req;
            if (gd.fixed_level >= 0) lev_req = gd.fixed_level;
            else if (gd.per_block) lev_req = P.block_level[c >> gd.block_shift];
            else lev_req = glevel;
            const bool enc = use;
            // subnormal flag of the group (wave ballots meet in LDS); not needed
            // at level 0, nor after a fused run whose truncation steps tested
            // every touched chunk and found none (uniform over the workgroup)
            uint32_t gs = 0;
            if (!verified && !(gd.fixed_level < 0 && !gd.per_block && glevel == 0)) {
                const bool wsub = __any(enc && sub);
                if ((tid & 63) == 0) slS[tid >> 6] = wsub ? 1u : 0u;
                lds_barrier();
#pragma unroll
                for (int i = 0; i < WPG; ++i) gs |= slS[s * WPG + i];
            }
            const bool gsub = gs != 0;
            // Sec. 3.8 per chunk (per-block levels): delta(level) * |v|^2 before
            // truncation, and the squared norm the truncation removes
            double pre = 0.0;
            if (DST == DST_ARENA && gd.per_block) {
#pragma unroll
                for (int k = 0; k < V; ++k) {
                    const double x = vals[vpos(first + k)];
                    pre += x * x;
                }
            }
            EncPlan<V> e;
            encode_plan<V, WPG, ENT>(xh, xl, xprev_hi, x0, x1, lev_req, gsub, C, lt, slE, slF, e, ent_on, b, ent, slD,
                                     rsh);
            if (DST == DST_ARENA && gd.per_block && enc) {
                double post = 0.0;
#pragma unroll
                for (int k = 0; k < V; ++k) {
                    const double t = u2d(((uint64_t)e.th[k] << 32) | e.tl[k]);
                    post += t * t;
                }
                acc_wd += level_delta(lev_req) * pre;
                acc_lost += pre - post;
            }
            // a sweep moves every chunk to the other arena: one the gate leaves
            // unchanged (skipped by its controls or its phases) is copied as it is
            const bool carry = DST == DST_ARENA && GATE && gd.sweep && valid && !act && ok_src;
            const uint32_t new_size = enc ? e.size : (uint32_t)(old_entry & 0xFFFFull);
            // claim arena space now; the returned offset is first needed after
            // the stream has been assembled in LDS, which hides the atomic
            uint64_t my_off = 0;
            const int stripe = (int)(blockIdx.x % (uint32_t)ds_nstripes);
            if (lt == 0 && (enc || carry) && DST == DST_ARENA)
                my_off = atomicAdd((unsigned long long *)&ds->stripe[stripe][0], (unsigned long long)alloc_bytes(new_size));
            // no barrier before clearing b[]: every read of the decoded values
            // (and of the other slot's buffer) precedes the plan's last barrier
            const uint32_t words = (e.size + 3u) >> 2;
            if (enc) {
                uint4 *b4 = reinterpret_cast<uint4 *>(b);   // 16-byte aligned; kBufWords % 4 == 0
                for (uint32_t w = lt; w < (words + 3u) >> 2; w += G) b4[w] = make_uint4(0u, 0u, 0u, 0u);
            }
            lds_barrier();
            if (enc) encode_emit<V>(b, e, C, lt, ent);
            if (lt == 0) {
                int ok = 0;
                if (enc || carry) {
                    if (DST == DST_ARENA) {
                        ok = (my_off + alloc_bytes(new_size) <= ds_ssize) ? 1 : 0;
                        my_off += ds_base + (uint64_t)stripe * ds_ssize;
                        if (!ok) atomicExch(&ds->fail, 1);
                    } else {
                        ok = 1;
                    }
                }
                sh_off[s] = my_off;
                sh_ok[s] = ok;
            }
            lds_barrier();
            const int ok = sh_ok[s];
            if (ok) {
                if (DST == DST_ARENA && carry) {
                    // the old stream, word by word (a compacted stream may start at any
                    // word), with its last 16-byte unit's tail cleared
                    const uint64_t offw = sh_off[s] >> 2, srcw = old_entry >> 16;
                    const uint32_t cw = (new_size + 3u) >> 2, units = (cw + 3u) >> 2;
                    for (uint32_t w = lt; w < 4u * units; w += G) P.out[offw + w] = w < cw ? P.arena[srcw + w] : 0u;
                } else if (DST == DST_ARENA) {
                    // whole 16-byte units: the allocation holds them and b[] is zero past the stream
                    const uint64_t offw = sh_off[s] >> 2;
                    u32x4 *dst4 = reinterpret_cast<u32x4 *>(P.out + offw);
                    const u32x4 *b4 = reinterpret_cast<const u32x4 *>(b);
                    for (uint32_t w = lt; w < (words + 3u) >> 2; w += G) dst4[w] = b4[w];
                } else {
                    for (uint32_t w = lt; w < words; w += G) io.slots_out[item * io.slot_words + w] = b[w];
                }
            }
            if (lt == 0 && valid) {
                if (DST == DST_ARENA) {
                    P.undo[item] = old_entry;
                    const uint64_t old_pad = ((old_entry & 0xFFFFull) + 3ull) & ~3ull;
                    const uint64_t new_pad = ((uint64_t)e.size + 3ull) & ~3ull;
                    // the size change counts also where the allocation failed: the
                    // gate's logged size is then its true one, which the budget
                    // test takes before the full arena
                    if (enc) sh_acc[4 * s] += new_pad - old_pad;   // two's complement: a signed delta
                    if (ok && carry) {
                        P.table[c] = ((sh_off[s] >> 2) << 16) | (uint64_t)new_size;
                    } else if (ok) {
                        P.table[c] = ((sh_off[s] >> 2) << 16) | (uint64_t)e.size;
                        sh_acc[4 * s + 1] += 1;
                        sh_acc[4 * s + 2] += old_pad;
                        sh_acc[4 * s + 3] += new_pad;
                    }
                } else {
                    io.sizes_out[item] = ok ? e.size : 0u;
                }
            }
        }
        lds_barrier();
    }

    if (DST == DST_MOMENTS) {
        // workgroup reduction of the three sums
        double a = mom_re, bb = mom_im, cc = mom_n2;
        for (int d = 32; d >= 1; d >>= 1) {
            a += __shfl_down(a, d, 64);
            bb += __shfl_down(bb, d, 64);
            cc += __shfl_down(cc, d, 64);
        }
        if ((tid & 63) == 0) { sh_mom[tid >> 6][0] = a; sh_mom[tid >> 6][1] = bb; sh_mom[tid >> 6][2] = cc; }
        lds_barrier();
        if (tid == 0) {
            double A = 0, B = 0, Cc = 0;
            for (int w = 0; w < WGS / 64; ++w) { A += sh_mom[w][0]; B += sh_mom[w][1]; Cc += sh_mom[w][2]; }
            io.partials[4 * blockIdx.x] = A;
            io.partials[4 * blockIdx.x + 1] = B;
            io.partials[4 * blockIdx.x + 2] = Cc;
            io.partials[4 * blockIdx.x + 3] = 0.0;
        }
    }

    if (DST == DST_ARENA) {
        constexpr int NRED = LIST == 2 ? 6 : 5;   // per-wavefront sums in the closing reduction
        // per-workgroup totals, then the last workgroup closes the gate
        if (gd.per_block) {
            double a = acc_wd, l = acc_lost;
            for (int d = 32; d >= 1; d >>= 1) {
                a += __shfl_down(a, d, 64);
                l += __shfl_down(l, d, 64);
            }
            if ((tid & 63) == 0) { sh_mom[tid >> 6][0] = a; sh_mom[tid >> 6][1] = l; }
        }
        lds_barrier();
        if (tid == 0) {
            WgPart wp;
            wp.delta = sh_acc[0] + sh_acc[4];
            wp.reenc = sh_acc[1] + sh_acc[5];
            wp.rd = sh_acc[2] + sh_acc[6];
            wp.wr = sh_acc[3] + sh_acc[7];
            wp.wd = 0.0;
            wp.lost = 0.0;
            if (gd.per_block)
                for (int w = 0; w < WGS / 64; ++w) { wp.wd += sh_mom[w][0]; wp.lost += sh_mom[w][1]; }
            wp.hits = 0;
            if (LIST == 1) {
                P.wgp[kMaxGrid / 2 + blockIdx.x] = wp;   // summed by the followers' launch
            } else {
                P.wgp[blockIdx.x] = wp;
                __threadfence();
                const uint32_t prev = atomicAdd(&ds->done, 1u);
                sh_ok[0] = (prev == gridDim.x - 1) ? 1 : 0;
            }
        }
        if (LIST == 1) return;
        lds_barrier();
        if (sh_ok[0]) {
            // the last workgroup: sum the partials of all workgroups
            __threadfence();
            uint64_t d = 0, r = 0, rd = 0, wr = 0, used = 0, h = 0;
            double fw = 0.0, fl = 0.0;
            for (uint32_t g = (uint32_t)tid; g < gridDim.x; g += WGS) {
                const WgPart wp = P.wgp[g];
                d += wp.delta;
                r += wp.reenc;
                rd += wp.rd;
                wr += wp.wr;
                fw += wp.wd;
                fl += wp.lost;
                if (LIST == 2) {   // the leaders' launch ran with the same grid
                    const WgPart wq = P.wgp[kMaxGrid / 2 + g];
                    d += wq.delta;
                    r += wq.reenc;
                    rd += wq.rd;
                    wr += wq.wr;
                }
            }
            if (LIST == 2)   // the followers' copy kernel (kCopyGrid workgroups)
                for (uint32_t g = (uint32_t)tid; g < (uint32_t)kCopyGrid; g += WGS) {
                    const WgPart wq = io.cparts[g];
                    d += wq.delta;
                    r += wq.reenc;
                    rd += wq.rd;
                    wr += wq.wr;
                    h += wq.hits;
                }
            if (tid < kStripes) used = atomicAdd((unsigned long long *)&ds->stripe[tid][0], 0ull);
            for (int off = 32; off >= 1; off >>= 1) {
                d += __shfl_down(d, off, 64);
                r += __shfl_down(r, off, 64);
                rd += __shfl_down(rd, off, 64);
                wr += __shfl_down(wr, off, 64);
                used += __shfl_down(used, off, 64);
                fw += __shfl_down(fw, off, 64);
                fl += __shfl_down(fl, off, 64);
                if (LIST == 2) h += __shfl_down(h, off, 64);
            }
            if ((tid & 63) == 0) { sh_mom[tid >> 6][2] = fw; sh_mom[tid >> 6][3] = fl; }
            uint64_t *red = reinterpret_cast<uint64_t *>(buf[0]);
            if ((tid & 63) == 0) {
                red[NRED * (tid >> 6)] = d;
                red[NRED * (tid >> 6) + 1] = r;
                red[NRED * (tid >> 6) + 2] = rd;
                red[NRED * (tid >> 6) + 3] = wr;
                red[NRED * (tid >> 6) + 4] = used;
                if (LIST == 2) red[NRED * (tid >> 6) + 5] = h;
            }
        }
        lds_barrier();
        if (tid == 0 && sh_ok[0]) {
            const uint64_t *red = reinterpret_cast<const uint64_t *>(buf[0]);
            uint64_t d = 0, r = 0, rd = 0, wr = 0, used = 0, h = 0;
            for (int w = 0; w < WGS / 64; ++w) {
                d += red[NRED * w];
                r += red[NRED * w + 1];
                rd += red[NRED * w + 2];
                wr += red[NRED * w + 3];
                used += red[NRED * w + 4];
                if (LIST == 2) h += red[NRED * w + 5];
            }
            const uint64_t live = ds->live + d;
            ds->live = live;
            GateLog lg;
            lg.live = live;
            lg.bump = ds->base + used;
            lg.reenc = r;
            lg.rd = rd;
            lg.wr = wr;
            lg.wd = 0.0;
            lg.lost = 0.0;
            for (int w = 0; w < WGS / 64; ++w) { lg.wd += sh_mom[w][2]; lg.lost += sh_mom[w][3]; }
            lg.hits = h;
            ds->log[gd.seq] = lg;
            const int fail = atomicExch(&ds->fail, 0);
            const int corrupt = atomicExch(&ds->corrupt, 0);
            int reason = STOP_NONE;
            // over the budget first: Sec. 3.7 relaxes the level whatever the arena holds
            if (corrupt) reason = STOP_CORRUPT;
            else if (ds->budget && live > ds->budget) reason = STOP_BUDGET;
            else if (fail) reason = STOP_ARENA;
            if (reason != STOP_NONE) {
                ds->stop_reason = reason;
                ds->stop_seq = gd.seq;
                __threadfence();
                ds->stop = 1;
            }
            atomicExch(&ds->done, 0u);
        }
    }
}

// ---------------------------------------------------------------------------
// chunk-group runs
// ---------------------------------------------------------------------------
// A run of chunk-pair gates (Sec. 3.3's pair update) whose targets are two
// chunk-index bits B1 = gd.pair_bit and B2 = gd.pair_bit2: a job is the group
// of four chunks base | {0, B1, B2, B1|B2}.  The two slots of the workgroup
// fetch and decode them in two rounds into four LDS buffers; each gate of the
// run updates the pairs it joins across the buffers, followed by the
// truncation its re-encoding would apply to the chunks it touched (none for a
// chunk holding a subnormal value); the two slots encode the four chunks in
// two rounds.  A chunk that no gate of the run touches keeps its stream (or is
// copied as it is in a sweep).  Bytes equal the gate-by-gate method's.
// C = 2048 only (V = 16, two wavefronts per chunk); not with the entropy stage.
__device__ __forceinline__ bool group_gate_touches(uint64_t cm, uint64_t c, int cb)
{
    return ((c << cb) & cm & ~(((uint64_t)1 << cb) - 1)) == (cm & ~(((uint64_t)1 << cb) - 1));
}

// V values per thread: a chunk slot is kCMax / V threads.  NB chunk-index bits
// per group (2 or 3): 2^NB chunks, 2^(NB-1) slots, each slot taking two of them.
template <int V, int NB>
__global__ __launch_bounds__((1 << (NB - 1)) * kCMax / V, NB == 2 ? 2 : 1) void group_kernel(GateDesc gd, DevPtrs P,
                                                                                             IOPtrs io)
{
    constexpr int NG = 1 << NB;        // chunks per group
    constexpr int NS = NG / 2;         // slots
    constexpr int G = kCMax / V;       // threads per chunk slot
    constexpr int WPG = G / 64;        // wavefronts per slot
    constexpr int WGS = NS * G;
    constexpr int NW = WGS / 64;       // wavefronts per workgroup
    static_assert(NW >= NG, "sh_sub also holds one flag per chunk of the group");
    __shared__ __align__(16) uint32_t buf[NG][kBufWords];
    __shared__ uint32_t sh[256];
    __shared__ uint64_t sh_off[NS];
    __shared__ int sh_ok[NS];
    __shared__ int sh_src_ok[NG];
    __shared__ uint64_t sh_acc[4 * NS];
    __shared__ double sh_rm[kMaxRun][8];
    __shared__ uint32_t sh_sub[2][NW];
    // the run's gates as the job loop reads them: control mask, and kind |
    // group index bit of the target << 8 (read from LDS: global reads inside
    // the job loop would be vector loads, each waited for on its own)
    __shared__ uint64_t sh_gcm[kMaxRun];
    __shared__ int32_t sh_gk[kMaxRun];

    DevState *ds = P.ds;
    if (ds->stop) return;
    const int tid = threadIdx.x, s = tid / G, lt = tid % G;
    for (int i = tid; i < 8 * io.nrun; i += WGS) sh_rm[i >> 3][i & 7] = io.run[i >> 3].m[i & 7];
    for (int r = tid; r < io.nrun; r += WGS) {
        sh_gcm[r] = io.run[r].cm;
        const uint64_t pb = io.run[r].pair_bit;
        sh_gk[r] = io.run[r].kind | ((pb == gd.pair_bit ? 1 : pb == gd.pair_bit2 ? 2 : 4) << 8);
    }
    const int C = P.C, cb = P.cb, ca = C / 2;
    const int first = lt * V;
    uint32_t *slA = sh, *slB = sh + 16, *slC = sh + 32, *slE = sh + 48, *slF = sh + 176, *slS = sh + 192;
    const int glevel = ds->level;
    const uint64_t ds_nstripes = ds->nstripes, ds_base = ds->base, ds_ssize = ds->stripe_size;
    const uint32_t mh = sig_mask_hi(sig_bits(glevel));
    if (lt == 0)
        for (int k = 0; k < 4; ++k) sh_acc[4 * s + k] = 0;
    int ntr = 0;   // truncation steps so far (alternating flag sets)
    lds_barrier();   // (the run's matrices and records)
    // the table entries of my two chunks of the next group, read while the
    // current group is decoded (no other workgroup writes them in this launch)
    uint64_t next_entry[2] = {0, 0};
    bool have_next = false;

    for (uint64_t job = job_begin(gd) + blockIdx.x; job < job_stop(gd); job += gridDim.x) {
        // the group's chunks and which of them some gate of the run touches
        uint64_t cg[NG];
        bool tg[NG];
        const uint64_t base = deposit(gd, job);
        // (lane r of every wavefront tests gate r: at most 64 gates per run)
        const int ln = tid & 63;
        const bool in_run = ln < io.nrun;
        const uint64_t lcm = sh_gcm[in_run ? ln : 0];
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            cg[g] = base | ((g & 1) ? gd.pair_bit : 0ull) | ((g & 2) ? gd.pair_bit2 : 0ull) |
                    ((g & 4) ? gd.pair_bit3 : 0ull);
            tg[g] = __ballot(in_run && group_gate_touches(lcm, cg[g], cb)) != 0;
        }
        // 1-2. fetch, decode and run; a second attempt when the first one met
        //      a subnormal value
        uint64_t old_entry[2] = {0, 0};
        bool ok_src_r[2] = {true, true};
        bool verified = false;   // the run's truncation steps found no subnormal value
        for (bool careful = false;; careful = true) {
            // 1. fetch the group's streams (each slot stages two, all loads in
            //    flight together), then decode them in two rounds
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int gi = NS * r + s;
                const uint64_t e = (have_next && !careful) ? next_entry[r] : P.table[cg[gi]];
                old_entry[r] = e;
                ok_src_r[r] = entry_ok(e, P.arena_words);
            }
            {
                // both streams' loads in flight together (16-byte aligned ones)
                const uint64_t e0 = old_entry[0], e1 = old_entry[1];
                const bool on0 = tg[s] && ok_src_r[0], on1 = tg[NS + s] && ok_src_r[1];
                const uint32_t w0 = ((uint32_t)(e0 & 0xFFFFull) + 3u) >> 2, w1 = ((uint32_t)(e1 & 0xFFFFull) + 3u) >> 2;
                const uint64_t off0 = e0 >> 16, off1 = e1 >> 16;
                if (((off0 | off1) & 3ull) == 0) {
                    stage_units2<G>(buf[s], P.arena + off0, w0, on0, buf[NS + s], P.arena + off1, w1, on1, lt);
                } else {
                    if (on0) stage_words<G>(buf[s], P.arena + off0, w0, lt);
                    if (on1) stage_words<G>(buf[NS + s], P.arena + off1, w1, lt);
                }
            }
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int gi = NS * r + s;
                if ((tg[gi] || gd.sweep) && !ok_src_r[r] && lt == 0) atomicExch(&ds->corrupt, 1);
                if (lt == 0) sh_src_ok[gi] = ok_src_r[r] ? 1 : 0;
            }
            if (!careful) {
                // the next group's entries (their loads complete during the decode)
                const uint64_t nj = job + gridDim.x;
                have_next = nj < job_stop(gd);
                if (have_next) {
                    const uint64_t nbase = deposit(gd, nj);
#pragma unroll
                    for (int r = 0; r < 2; ++r) {
                        const int gi = NS * r + s;
                        const uint64_t c = nbase | ((gi & 1) ? gd.pair_bit : 0ull) | ((gi & 2) ? gd.pair_bit2 : 0ull) |
                                           ((gi & 4) ? gd.pair_bit3 : 0ull);
                        next_entry[r] = P.table[c];
                    }
                }
            }
            lds_barrier();
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int gi = NS * r + s;
                uint32_t *b = buf[gi];
                double *vals = reinterpret_cast<double *>(b);
                // the round's streams: mine, and whether any slot holds a SPARSE
                // or a Solution D stream (branches with barriers: uniform)
                bool use = false, any_sparse = false, any_rsh = false;
                uint32_t my_hdr = (uint32_t)M_CONST2;
#pragma unroll
                for (int j = 0; j < NS; ++j) {
                    const int gj = NS * r + j;
                    const bool uj = tg[gj] && sh_src_ok[gj] != 0;
                    const uint32_t hj = uj ? buf[gj][0] : (uint32_t)M_CONST2;
                    any_sparse = any_sparse || (hj & 3u) == M_SPARSE;
                    any_rsh = any_rsh || (uj && (hj & kHdrRsh) != 0);
                    if (j == s) {
                        use = uj;
                        my_hdr = hj;
                    }
                }
                uint32_t th[V], tl[V];
                decode_group<V, WPG, false>(b, my_hdr, use, any_sparse, C, lt, slA, slB, slC, th, tl);
                lds_barrier();
                double x[V];
#pragma unroll
                for (int k = 0; k < V; ++k) x[k] = u2d(((uint64_t)th[k] << 32) | tl[k]);
                if (any_rsh) {
                    const bool mine = use && (my_hdr & kHdrRsh) != 0;
#pragma unroll
                    for (int k = 0; k < V; ++k) vals[vpos(mine ? rsh_pos(first + k, C) : first + k)] = x[k];
                    lds_barrier();
#pragma unroll
                    for (int k = 0; k < V; ++k) x[k] = vals[vpos(first + k)];
                }
#pragma unroll
                for (int k = 0; k < V; ++k) vals[vpos(first + k)] = x[k];
                lds_barrier();
            }

            // 2. the run: each gate on the pairs it joins, then its truncation,
            //    none for a chunk holding a subnormal value.  The first attempt
            //    truncates each value as the gate writes it and notes whether a
            //    touched value came out subnormal; if one did, the group is
            //    fetched and run again, deciding over each whole chunk after
            //    every gate.
            const bool inline_trunc = !careful && glevel > 0;
            bool seen = false;   // a value I truncated came out subnormal
            for (int r = 0; r < io.nrun; ++r) {
                const uint64_t rcm = uni64(sh_gcm[r]);
                const int32_t rk = uni32(sh_gk[r]);
                const int rkind = rk & 0xFF, bitsel = rk >> 8;   // group index bit of the target
                const uint32_t cm_lo = (uint32_t)(rcm & (uint64_t)(ca - 1));
                // pair q (0 .. NS-1): group indices p0 < p1 differing in bitsel,
                // p0 the q-th index with that bit clear
                const int bpos = bitsel == 1 ? 0 : bitsel == 2 ? 1 : 2;
                bool pact[NS];
                int pg0[NS], pg1[NS];
                bool any_pact = false;
#pragma unroll
                for (int q = 0; q < NS; ++q) {
                    pg0[q] = ((q >> bpos) << (bpos + 1)) | (q & (bitsel - 1));
                    pg1[q] = pg0[q] | bitsel;
                    pact[q] = tg[pg0[q]] && tg[pg1[q]] && sh_src_ok[pg0[q]] && sh_src_ok[pg1[q]] &&
                              group_gate_touches(rcm, cg[pg0[q]], cb);
                    any_pact = any_pact || pact[q];
                }
                {
                    const int q = tid / G;   // the slot's threads take pair q
                    if (pact[q]) {
                        double *v0 = reinterpret_cast<double *>(buf[pg0[q]]);
                        double *v1 = reinterpret_cast<double *>(buf[pg1[q]]);
                        const double u0r = sh_rm[r][0], u0i = sh_rm[r][1], u1r = sh_rm[r][2], u1i = sh_rm[r][3];
                        const double u2r = sh_rm[r][4], u2i = sh_rm[r][5], u3r = sh_rm[r][6], u3i = sh_rm[r][7];
                        for (int k = tid % G; k < ca; k += G) {
                            const bool on = ((uint32_t)k & cm_lo) == cm_lo;
                            if (!on && !inline_trunc) continue;
                            const int p = vpos(2 * k);
                            double ar = v0[p], ai = v0[p + 1], br = v1[p], bi = v1[p + 1];
                            if (on) {
                                if (rkind == K_X) {
                                    const double tr = ar, ti = ai;
                                    ar = br; ai = bi; br = tr; bi = ti;
                                } else {
                                    double yr, yi, zr, zi;
                                    lin2(u0r, u0i, u1r, u1i, ar, ai, br, bi, yr, yi);
                                    lin2(u2r, u2i, u3r, u3i, ar, ai, br, bi, zr, zi);
                                    ar = yr; ai = yi; br = zr; bi = zi;
                                }
                            }
                            if (inline_trunc) {
                                seen = seen || is_subnormal(ar) || is_subnormal(ai) || is_subnormal(br) || is_subnormal(bi);
                                ar = u2d((uint64_t)((uint32_t)(d2u(ar) >> 32) & mh) << 32);
                                ai = u2d((uint64_t)((uint32_t)(d2u(ai) >> 32) & mh) << 32);
                                br = u2d((uint64_t)((uint32_t)(d2u(br) >> 32) & mh) << 32);
                                bi = u2d((uint64_t)((uint32_t)(d2u(bi) >> 32) & mh) << 32);
                            }
                            v0[p] = ar; v0[p + 1] = ai; v1[p] = br; v1[p + 1] = bi;
                        }
                    }
                }
                lds_barrier();
                if (careful && glevel > 0 && any_pact) {
                    // per touched chunk: a subnormal value anywhere keeps it untruncated
                    uint32_t *flags = sh_sub[ntr & 1];
                    if (tid < NG) flags[tid] = 0u;
                    lds_barrier();
#pragma unroll
                    for (int g = 0; g < NG; ++g) {
                        bool touched = false;
#pragma unroll
                        for (int q = 0; q < NS; ++q) touched = touched || (pact[q] && (g == pg0[q] || g == pg1[q]));
                        if (!touched) continue;
                        const double *v = reinterpret_cast<const double *>(buf[g]);
                        bool sub = false;
                        for (int i = tid; i < C; i += WGS) {
                            const uint64_t u = d2u(v[vpos(i)]);
                            sub = sub || subnormal((uint32_t)(u >> 32), (uint32_t)u);
                        }
                        if (__any(sub) && (tid & 63) == 0) atomicOr(&flags[g], 1u);
                    }
                    lds_barrier();
#pragma unroll
                    for (int g = 0; g < NG; ++g) {
                        bool touched = false;
#pragma unroll
                        for (int q = 0; q < NS; ++q) touched = touched || (pact[q] && (g == pg0[q] || g == pg1[q]));
                        if (!touched || flags[g]) continue;
                        double *v = reinterpret_cast<double *>(buf[g]);
                        for (int i = tid; i < C; i += WGS) {
                            const int p = vpos(i);
                            v[p] = u2d((uint64_t)((uint32_t)(d2u(v[p]) >> 32) & mh) << 32);
                        }
                    }
                    ++ntr;
                    lds_barrier();
                }
            }
            if (inline_trunc) {
                // (sh_sub is next written after the fetch barrier of the second
                // attempt or of a later job)
                const bool wsub = __any(seen);
                if ((tid & 63) == 0) sh_sub[0][tid >> 6] = wsub ? 1u : 0u;
                lds_barrier();
                uint32_t any = 0;
#pragma unroll
                for (int i = 0; i < NW; ++i) any |= sh_sub[0][i];
                if (any != 0) continue;   // (uniform over the workgroup)
                verified = true;
            }
            break;
        }

        // 3. two rounds of encode, claim and copy-out
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int gi = NS * r + s;
            uint32_t *b = buf[gi];
            const double *vals = reinterpret_cast<const double *>(b);
            const uint64_t c = cg[gi];
            const uint64_t item = (uint64_t)NG * job + (uint64_t)gi;
            const bool use = tg[gi] && sh_src_ok[gi] != 0;
            const bool carry = gd.sweep && !tg[gi] && ok_src_r[r];
            uint32_t xh[V], xl[V];
            bool sub = false;
            const bool rsh = gd.reshuffle != 0;
#pragma unroll
            for (int k = 0; k < V; ++k) {
                const uint64_t x = d2u(vals[vpos(rsh ? rsh_pos(first + k, C) : first + k)]);
                xh[k] = (uint32_t)(x >> 32);
                xl[k] = (uint32_t)x;
                sub = sub || subnormal(xh[k], xl[k]);
            }
            const uint32_t xprev_hi =
                lt ? (uint32_t)(d2u(vals[vpos(rsh ? rsh_pos(first - 1, C) : first - 1)]) >> 32) : 0u;
            const uint64_t x0 = d2u(vals[0]), x1 = d2u(vals[1]);
            // subnormal flag of the chunk: not needed at level 0, nor when the
            // run's truncation steps tested every touched chunk and found none
            uint32_t gs = 0;
            if (!verified && glevel > 0) {
                const bool wsub = __any(use && sub);
                if ((tid & 63) == 0) slS[tid >> 6] = wsub ? 1u : 0u;
                lds_barrier();
#pragma unroll
                for (int i = 0; i < WPG; ++i) gs |= slS[s * WPG + i];
            }
            EncPlan<V> e;
            encode_plan<V, WPG, false>(xh, xl, xprev_hi, x0, x1, glevel, gs != 0, C, lt, slE, slF, e, false, nullptr,
                                       nullptr, nullptr, rsh);
            const uint32_t new_size = use ? e.size : (uint32_t)(old_entry[r] & 0xFFFFull);
            uint64_t my_off = 0;
            const int stripe = (int)(blockIdx.x % (uint32_t)ds_nstripes);
            if (lt == 0 && (use || carry))
                my_off = atomicAdd((unsigned long long *)&ds->stripe[stripe][0], (unsigned long long)alloc_bytes(new_size));
            const uint32_t words = (e.size + 3u) >> 2;
            if (use) {
                uint4 *b4 = reinterpret_cast<uint4 *>(b);
                for (uint32_t w = lt; w < (words + 3u) >> 2; w += G) b4[w] = make_uint4(0u, 0u, 0u, 0u);
            }
            lds_barrier();
            if (use) encode_emit<V>(b, e, C, lt);
            if (lt == 0) {
                int ok = 0;
                if (use || carry) {
                    ok = (my_off + alloc_bytes(new_size) <= ds_ssize) ? 1 : 0;
                    my_off += ds_base + (uint64_t)stripe * ds_ssize;
                    if (!ok) atomicExch(&ds->fail, 1);
                }
                sh_off[s] = my_off;
                sh_ok[s] = ok;
            }
            lds_barrier();
            const int ok = sh_ok[s];
            if (ok && carry) {
                const uint64_t offw = sh_off[s] >> 2, srcw = old_entry[r] >> 16;
                const uint32_t cw = (new_size + 3u) >> 2, units = (cw + 3u) >> 2;
                for (uint32_t w = lt; w < 4u * units; w += G) P.out[offw + w] = w < cw ? P.arena[srcw + w] : 0u;
            } else if (ok) {
                const uint64_t offw = sh_off[s] >> 2;
                u32x4 *dst4 = reinterpret_cast<u32x4 *>(P.out + offw);
                const u32x4 *b4 = reinterpret_cast<const u32x4 *>(b);
                for (uint32_t w = lt; w < (words + 3u) >> 2; w += G) dst4[w] = b4[w];
            }
            if (lt == 0) {
                P.undo[item] = old_entry[r];
                const uint64_t old_pad = ((old_entry[r] & 0xFFFFull) + 3ull) & ~3ull;
                const uint64_t new_pad = ((uint64_t)e.size + 3ull) & ~3ull;
                if (use) sh_acc[4 * s] += new_pad - old_pad;   // (also where the claim failed)
                if (ok && carry) {
                    P.table[c] = ((sh_off[s] >> 2) << 16) | (uint64_t)new_size;
                } else if (ok) {
                    P.table[c] = ((sh_off[s] >> 2) << 16) | (uint64_t)e.size;
                    sh_acc[4 * s + 1] += 1;
                    sh_acc[4 * s + 2] += old_pad;
                    sh_acc[4 * s + 3] += new_pad;
                }
            }
            lds_barrier();
        }
    }

    // per-workgroup totals; the last workgroup closes the run
    if (tid == 0) {
        WgPart wp;
        wp.delta = wp.reenc = wp.rd = wp.wr = 0;
        for (int j = 0; j < NS; ++j) {
            wp.delta += sh_acc[4 * j];
            wp.reenc += sh_acc[4 * j + 1];
            wp.rd += sh_acc[4 * j + 2];
            wp.wr += sh_acc[4 * j + 3];
        }
        wp.wd = 0.0;
        wp.lost = 0.0;
        wp.hits = 0;
        P.wgp[blockIdx.x] = wp;
        __threadfence();
        const uint32_t prev = atomicAdd(&ds->done, 1u);
        sh_ok[0] = (prev == gridDim.x - 1) ? 1 : 0;
    }
    lds_barrier();
    if (sh_ok[0]) {
        __threadfence();
        uint64_t d = 0, rr = 0, rd = 0, wr = 0, used = 0;
        for (uint32_t g = (uint32_t)tid; g < gridDim.x; g += WGS) {
            const WgPart wp = P.wgp[g];
            d += wp.delta;
            rr += wp.reenc;
            rd += wp.rd;
            wr += wp.wr;
        }
        if (tid < kStripes) used = atomicAdd((unsigned long long *)&ds->stripe[tid][0], 0ull);
        for (int off = 32; off >= 1; off >>= 1) {
            d += __shfl_down(d, off, 64);
            rr += __shfl_down(rr, off, 64);
            rd += __shfl_down(rd, off, 64);
            wr += __shfl_down(wr, off, 64);
            used += __shfl_down(used, off, 64);
        }
        uint64_t *red = reinterpret_cast<uint64_t *>(buf[0]);
        if ((tid & 63) == 0) {
            red[5 * (tid >> 6)] = d;
            red[5 * (tid >> 6) + 1] = rr;
            red[5 * (tid >> 6) + 2] = rd;
            red[5 * (tid >> 6) + 3] = wr;
            red[5 * (tid >> 6) + 4] = used;
        }
    }
    lds_barrier();
    if (tid == 0 && sh_ok[0]) {
        const uint64_t *red = reinterpret_cast<const uint64_t *>(buf[0]);
        uint64_t d = 0, rr = 0, rd = 0, wr = 0, used = 0;
        for (int w = 0; w < WGS / 64; ++w) {
            d += red[5 * w];
            rr += red[5 * w + 1];
            rd += red[5 * w + 2];
            wr += red[5 * w + 3];
            used += red[5 * w + 4];
        }
        const uint64_t live = ds->live + d;
        ds->live = live;
        GateLog lg;
        lg.live = live;
        lg.bump = ds->base + used;
        lg.reenc = rr;
        lg.rd = rd;
        lg.wr = wr;
        lg.wd = 0.0;
        lg.lost = 0.0;
        lg.hits = 0;
        ds->log[gd.seq] = lg;
        const int fail = atomicExch(&ds->fail, 0);
        const int corrupt = atomicExch(&ds->corrupt, 0);
        int reason = STOP_NONE;
        if (corrupt) reason = STOP_CORRUPT;
        else if (ds->budget && live > ds->budget) reason = STOP_BUDGET;
        else if (fail) reason = STOP_ARENA;
        if (reason != STOP_NONE) {
            ds->stop_reason = reason;
            ds->stop_seq = gd.seq;
            __threadfence();
            ds->stop = 1;
        }
        atomicExch(&ds->done, 0u);
    }
}

// X on chunk-index bits with no control inside the chunk: exchange table
// entries (the streams themselves are unchanged and exact).
__global__ __launch_bounds__(kWG) void permute_kernel(GateDesc gd, DevPtrs P)
{
    __shared__ int last;
    DevState *ds = P.ds;
    if (ds->stop) return;
    const uint64_t stride = (uint64_t)gridDim.x * kWG;
    for (uint64_t j = (uint64_t)blockIdx.x * kWG + threadIdx.x; j < gd.njobs; j += stride) {
        const uint64_t c0 = deposit(gd, j), c1 = c0 | gd.pair_bit;
        const uint64_t e0 = P.table[c0], e1 = P.table[c1];
        P.table[c0] = e1;
        P.table[c1] = e0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const uint32_t prev = atomicAdd(&ds->done, 1u);
        last = (prev == gridDim.x - 1) ? 1 : 0;
    }
    __syncthreads();
    if (threadIdx.x == 0 && last) {
        __threadfence();
        GateLog lg;
        lg.live = ds->live;
        uint64_t used = 0;
        for (int k = 0; k < kStripes; ++k) used += atomicAdd((unsigned long long *)&ds->stripe[k][0], 0ull);
        lg.bump = ds->base + used;
        lg.reenc = 0;
        lg.rd = lg.wr = 0;
        lg.wd = lg.lost = 0.0;
        lg.hits = 0;
        ds->log[gd.seq] = lg;
        atomicExch(&ds->done, 0u);
    }
}

// undo one gate: restore the table entries recorded by its jobs
__global__ __launch_bounds__(kWG) void rollback_kernel(GateDesc gd, DevPtrs P)
{
    const uint64_t stride = (uint64_t)gridDim.x * kWG;
    if (gd.job_type == J_PERMUTE) {
        for (uint64_t j = (uint64_t)blockIdx.x * kWG + threadIdx.x; j < gd.njobs; j += stride) {
            const uint64_t c0 = deposit(gd, j), c1 = c0 | gd.pair_bit;
            const uint64_t e0 = P.table[c0], e1 = P.table[c1];
            P.table[c0] = e1;
            P.table[c1] = e0;
        }
        return;
    }
    // the items of jobs [job_begin, job_stop): two per job (four in chunk groups)
    const uint64_t ipj = items_per_job(gd);
    const uint64_t it0 = ipj * job_begin(gd);
    const uint64_t it1 = ipj * job_stop(gd) < gd.nitems ? ipj * job_stop(gd) : gd.nitems;
    for (uint64_t it = it0 + (uint64_t)blockIdx.x * kWG + threadIdx.x; it < it1; it += stride)
        P.table[item_chunk(gd, it)] = P.undo[it];
}

__global__ __launch_bounds__(kWG) void fill_table_kernel(uint64_t *table, uint64_t n, uint64_t e0, uint64_t erest)
{
    const uint64_t stride = (uint64_t)gridDim.x * kWG;
    for (uint64_t c = (uint64_t)blockIdx.x * kWG + threadIdx.x; c < n; c += stride) table[c] = c ? erest : e0;
}

// the finalizer of SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): a
// bijective 64-bit mix
__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Block cache (Sec. 3.4) of one gate launch, first pass: one wavefront per
// job hashes the job's input streams (word values with their positions, and
// the size) and the chunk-index bits the gate reads into a 64-bit key.  Jobs
// with no stream to re-encode, or with an entry outside the arena, get
// kEmptyKey: they lead without looking for a match.
__global__ __launch_bounds__(kWG) void cache_hash_kernel(GateDesc gd, DevPtrs P, CachePtrs cp)
{
    // clear the key table (read by the next kernel only)
    for (uint64_t i = (uint64_t)blockIdx.x * kWG + threadIdx.x; i < cp.tsize; i += (uint64_t)gridDim.x * kWG)
        cp.keys[i] = kEmptyKey;
    uint32_t unit_mask = 0;
    for (int i = 0; i < 4; ++i) unit_mask |= unit_phase(gd.m[2 * i], gd.m[2 * i + 1]) ? (1u << i) : 0u;
    const IOPtrs io = {};
    const uint64_t opm = op_mask(gd, P.cb);
    const int lane = (int)(threadIdx.x & 63);
    const uint64_t nw = (uint64_t)gridDim.x * (kWG / 64);
    const uint64_t j0 = job_begin(gd), j1 = job_stop(gd);
    for (uint64_t job = j0 + (uint64_t)blockIdx.x * (kWG / 64) + (threadIdx.x >> 6); job < j1; job += nw) {
        uint64_t key = 0x243F6A8885A308D3ull;
        bool work = false, plain = false;
        for (int sl = 0; sl < 2; ++sl) {
            const uint64_t item = 2 * job + (uint64_t)sl;
            uint64_t c = 0;
            const bool act = job_slot<SRC_ARENA, true>(gd, unit_mask, io, P.cb, item, c);
            const bool valid = item < gd.nitems;
            uint64_t h = 0;
            if (act) {
                const uint64_t e = P.table[c];
                if (entry_ok(e, P.arena_words)) {
                    const uint32_t size = (uint32_t)(e & 0xFFFFull), words = (size + 3u) >> 2;
                    const uint32_t *w = P.arena + (e >> 16);
                    for (uint32_t i0 = (uint32_t)lane; i0 < words; i0 += 8u * 64u) {   // eight loads in flight
                        uint32_t v[8];
#pragma unroll
                        for (int u = 0; u < 8; ++u) {
                            const uint32_t i = i0 + 64u * (uint32_t)u;
                            v[u] = i < words ? w[i] : 0u;
                        }
#pragma unroll
                        for (int u = 0; u < 8; ++u) {
                            const uint32_t i = i0 + 64u * (uint32_t)u;
                            h += i < words ? mix64(((uint64_t)i << 32) | v[u]) : 0ull;
                        }
                    }
                    for (int o = 32; o >= 1; o >>= 1) h += __shfl_xor(h, o, 64);
                    h = mix64(h ^ ((uint64_t)size << 40));
                    work = true;
                } else {
                    plain = true;
                }
            }
            const uint64_t tag = (c & opm) ^ ((uint64_t)(valid ? 1 : 0) << 62) ^ ((uint64_t)(act ? 1 : 0) << 63);
            key = mix64(key ^ h) + mix64(tag + (uint64_t)sl);
        }
        if (lane != 0) continue;
        if (work && !plain) {
            key &= cp.key_mask;
            if (key == kEmptyKey) key ^= 1ull;
        } else {
            key = kEmptyKey;
        }
        cp.jkey[job - j0] = key;
    }
}

// Second pass, one thread per job: jobs of a workgroup meet in an LDS table
// first, so that only one job per distinct key and workgroup inserts into the
// global open-addressing table.  The job that inserts a key globally leads
// (role 0); every other job with that key follows the slot's owner (role 1 +
// slot).
__global__ __launch_bounds__(kWG) void cache_dedupe_kernel(GateDesc gd, CachePtrs cp)
{
    __shared__ unsigned long long tkey[2 * kWG];
    __shared__ uint32_t town[2 * kWG];
    __shared__ uint32_t tslot[kWG];
    const int t = (int)threadIdx.x;
    tkey[t] = kEmptyKey;
    tkey[t + kWG] = kEmptyKey;
    __syncthreads();
    const uint64_t j0 = job_begin(gd), j1 = job_stop(gd);
    const uint64_t job = j0 + (uint64_t)blockIdx.x * kWG + (uint64_t)t;
    const uint64_t key = job < j1 ? cp.jkey[job - j0] : kEmptyKey;
    int h = -1;
    if (key != kEmptyKey) {
        int p = (int)((key >> 17) & (2 * kWG - 1));
        for (int probe = 0; probe < 2 * kWG; ++probe) {
            const unsigned long long prev = atomicCAS(&tkey[p], (unsigned long long)kEmptyKey, (unsigned long long)key);
            if (prev == kEmptyKey) { town[p] = (uint32_t)t; h = p; break; }
            if (prev == key) { h = p; break; }
            p = (p + 1) & (2 * kWG - 1);
        }
    }
    __syncthreads();
    const int lead = h >= 0 ? (int)town[h] : t;
    uint32_t role = 0;
    if (h >= 0 && lead == t) {   // the workgroup's first job with this key: global insert
        uint64_t slot = key & (cp.tsize - 1);
        for (uint64_t probe = 0; probe < cp.tsize; ++probe) {
            const uint64_t prev = atomicCAS((unsigned long long *)&cp.keys[slot], (unsigned long long)kEmptyKey,
                                            (unsigned long long)key);
            if (prev == kEmptyKey) {
                cp.owner[slot] = (uint32_t)job;
                break;
            }
            if (prev == key) {
                role = 1u + (uint32_t)slot;
                break;
            }
            slot = (slot + 1) & (cp.tsize - 1);
        }
        tslot[t] = (uint32_t)slot;
    }
    __syncthreads();
    if (h >= 0 && lead != t) role = 1u + tslot[lead];
    if (job < j1) cp.role[job - j0] = role;
}

// Block cache followers, one wavefront per job: when both positions hold the
// same streams as the leader job's inputs (byte comparison) and the gate reads
// the same index bits, copy the leader's new streams (written by the leaders'
// launch) and mark the job done; otherwise leave it to the followers' job
// launch, which computes it.  Many jobs are in flight per CU, so the chain of
// dependent loads of a follower is overlapped.  Per-workgroup sums go to
// `parts` (always written, kCopyGrid workgroups), closed by that launch.
__global__ __launch_bounds__(kWG) void cache_copy_kernel(GateDesc gd, DevPtrs P, CachePtrs cp, WgPart *parts)
{
    __shared__ uint64_t red[kWG / 64][5];
    uint32_t unit_mask = 0;
    for (int i = 0; i < 4; ++i) unit_mask |= unit_phase(gd.m[2 * i], gd.m[2 * i + 1]) ? (1u << i) : 0u;
    const IOPtrs io = {};
    const uint64_t opm = op_mask(gd, P.cb);
    const int lane = (int)(threadIdx.x & 63), wv = (int)(threadIdx.x >> 6);
    DevState *ds = P.ds;
    const uint64_t nstr = ds->nstripes, sbase = ds->base, ssize = ds->stripe_size;
    const int stripe = (int)(blockIdx.x % (uint32_t)nstr);
    uint64_t a_d = 0, a_r = 0, a_rd = 0, a_wr = 0, a_h = 0;   // lane 0 of each wavefront
    const uint64_t j0 = job_begin(gd), j1 = job_stop(gd);
    const uint64_t nw = (uint64_t)gridDim.x * (kWG / 64);
    const bool run = ds->stop == 0;
    for (uint64_t job = j0 + (uint64_t)blockIdx.x * (kWG / 64) + (uint64_t)wv; run && job < j1; job += nw) {
        const uint32_t role = cp.role[job - j0];
        if (role == 0u) continue;
        const uint64_t lj = cp.owner[role - 1u];
        uint64_t c[2], mine[2], lnew[2];
        bool act[2], valid[2], same = true;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const uint64_t item = 2 * job + (uint64_t)s, li = 2 * lj + (uint64_t)s;
            uint64_t lc = 0;
            act[s] = job_slot<SRC_ARENA, true>(gd, unit_mask, io, P.cb, item, c[s]);
            const bool lact = job_slot<SRC_ARENA, true>(gd, unit_mask, io, P.cb, li, lc);
            valid[s] = item < gd.nitems;
            const bool lvalid = li < gd.nitems;
            mine[s] = valid[s] ? P.table[c[s]] : 0ull;
            const uint64_t lold = lvalid ? P.undo[li] : 0ull;
            lnew[s] = act[s] ? P.table[lc] : 0ull;
            bool ss = valid[s] == lvalid && act[s] == lact && (c[s] & opm) == (lc & opm);
            if (ss && act[s])
                ss = (mine[s] & 0xFFFFull) == (lold & 0xFFFFull) && entry_ok(mine[s], P.arena_words) &&
                     entry_ok(lold, P.arena_words) && entry_ok(lnew[s], P.arena_words);
            if (ss && act[s]) {
                const uint32_t words = (uint32_t)(((mine[s] & 0xFFFFull) + 3ull) >> 2);
                const uint32_t *pa = P.arena + (mine[s] >> 16), *pb = P.arena + (lold >> 16);
                uint32_t diff = 0;
                for (uint32_t w = (uint32_t)lane; w < words; w += 64) diff |= pa[w] ^ pb[w];
                ss = !__any(diff != 0u);
            }
            same = same && ss;
        }
        if (!same) continue;   // computed by the followers' job launch
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const uint64_t item = 2 * job + (uint64_t)s;
            if (!act[s]) {
                if (valid[s] && lane == 0) P.undo[item] = mine[s];
                continue;
            }
            const uint32_t nsize = (uint32_t)(lnew[s] & 0xFFFFull);
            unsigned long long off = 0;
            if (lane == 0)
                off = atomicAdd((unsigned long long *)&ds->stripe[stripe][0], (unsigned long long)alloc_bytes(nsize));
            off = __shfl(off, 0, 64);
            const bool ok = off + alloc_bytes(nsize) <= ssize;
            if (ok) {
                const uint64_t dstw = (sbase + (uint64_t)stripe * ssize + off) >> 2, srcw = lnew[s] >> 16;
                const uint32_t words = (nsize + 3u) >> 2;
                if ((srcw & 3ull) == 0) {   // whole 16-byte units, zero past the leader's stream
                    const u32x4 *s4 = reinterpret_cast<const u32x4 *>(P.arena + srcw);
                    u32x4 *d4 = reinterpret_cast<u32x4 *>(P.arena + dstw);
                    for (uint32_t w = (uint32_t)lane; w < (words + 3u) >> 2; w += 64) d4[w] = s4[w];
                } else {
                    for (uint32_t w = (uint32_t)lane; w < ((words + 3u) & ~3u); w += 64)
                        P.arena[dstw + w] = w < words ? P.arena[srcw + w] : 0u;
                }
                if (lane == 0) {
                    P.table[c[s]] = (dstw << 16) | (uint64_t)nsize;
                    const uint64_t old_pad = ((mine[s] & 0xFFFFull) + 3ull) & ~3ull;
                    const uint64_t new_pad = ((uint64_t)nsize + 3ull) & ~3ull;
                    a_d += new_pad - old_pad;
                    a_r += 1;
                    a_rd += old_pad;
                    a_wr += new_pad;
                    a_h += 1;
                }
            } else if (lane == 0) {
                atomicExch(&ds->fail, 1);
            }
            if (lane == 0) P.undo[item] = mine[s];
        }
        if (lane == 0) cp.role[job - j0] = kRoleDone;
    }
    if (lane == 0) {
        red[wv][0] = a_d; red[wv][1] = a_r; red[wv][2] = a_rd; red[wv][3] = a_wr; red[wv][4] = a_h;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        WgPart wp = {};
        for (int w = 0; w < kWG / 64; ++w) {
            wp.delta += red[w][0]; wp.reenc += red[w][1]; wp.rd += red[w][2]; wp.wr += red[w][3]; wp.hits += red[w][4];
        }
        parts[blockIdx.x] = wp;
    }
}

// ---------------------------------------------------------------------------
// compaction: copy live chunks, in chunk order, into the other arena
// ---------------------------------------------------------------------------
constexpr int kScanItems = 1024;  // chunks per scan block

__global__ __launch_bounds__(kWG) void scan_local_kernel(const uint64_t *table, uint64_t n, uint64_t *excl,
                                                         uint64_t *block_sums)
{
    __shared__ uint64_t part[kWG];
    const uint64_t base = (uint64_t)blockIdx.x * kScanItems;
    uint64_t v[4], run = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint64_t c = base + 4 * threadIdx.x + k;
        v[k] = c < n ? (uint64_t)alloc_bytes((uint32_t)(table[c] & 0xFFFFull)) : 0ull;
        run += v[k];
    }
    part[threadIdx.x] = run;
    __syncthreads();
    for (int d = 1; d < kWG; d <<= 1) {
        uint64_t y = threadIdx.x >= (unsigned)d ? part[threadIdx.x - d] : 0ull;
        __syncthreads();
        part[threadIdx.x] += y;
        __syncthreads();
    }
    uint64_t pre = part[threadIdx.x] - run;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint64_t c = base + 4 * threadIdx.x + k;
        if (c < n) excl[c] = pre;
        pre += v[k];
    }
    if (threadIdx.x == kWG - 1) block_sums[blockIdx.x] = part[kWG - 1];
}

// single workgroup: exclusive scan of the block sums in place; total at [nb]
__global__ __launch_bounds__(kWG) void scan_blocks_kernel(uint64_t *block_sums, uint64_t nb)
{
    __shared__ uint64_t part[kWG];
    __shared__ uint64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (uint64_t base = 0; base < nb; base += kWG) {
        const uint64_t i = base + threadIdx.x;
        const uint64_t v = i < nb ? block_sums[i] : 0ull;
        part[threadIdx.x] = v;
        __syncthreads();
        for (int d = 1; d < kWG; d <<= 1) {
            uint64_t y = threadIdx.x >= (unsigned)d ? part[threadIdx.x - d] : 0ull;
            __syncthreads();
            part[threadIdx.x] += y;
            __syncthreads();
        }
        if (i < nb) block_sums[i] = carry + part[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 0) carry += part[kWG - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) block_sums[nb] = carry;
}

// one wavefront per chunk
__global__ __launch_bounds__(kWG) void compact_copy_kernel(DevPtrs P, uint32_t *dst, const uint64_t *excl,
                                                           const uint64_t *block_sums)
{
    const int lane = threadIdx.x & 63;
    const uint64_t wave = ((uint64_t)blockIdx.x * kWG + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * kWG) >> 6;
    for (uint64_t c = wave; c < P.nchunks; c += nwaves) {
        const uint64_t e = P.table[c];
        const uint32_t size = (uint32_t)(e & 0xFFFFull);
        const uint64_t off = e >> 16;
        const uint32_t words = (size + 3u) >> 2;
        const uint64_t noff = (block_sums[c / kScanItems] + excl[c]) >> 2;
        for (uint32_t w = lane; w < words; w += 64) dst[noff + w] = P.arena[off + w];
        if (lane == 0) P.table[c] = (noff << 16) | (uint64_t)size;
    }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
template <int V, int WPG, int SRC, int DST, bool GATE, bool ENT = false>
static void launch_vw(const GateDesc &gd, const DevPtrs &P, const IOPtrs &io, int grid, hipStream_t st,
                      hipEvent_t t0, hipEvent_t t1)
{
    if (t0) {  // events attached to the dispatch itself: they time exactly this kernel
        hipExtLaunchKernelGGL((job_kernel<V, WPG, SRC, DST, GATE, 0, ENT>), dim3(grid), dim3(128 * WPG), 0, st, t0, t1,
                              0, gd, P, io);
    } else {
        hipLaunchKernelGGL((job_kernel<V, WPG, SRC, DST, GATE, 0, ENT>), dim3(grid), dim3(128 * WPG), 0, st, gd, P,
                           io);
    }
}

// V values per thread and WPG wavefronts per chunk slot: C = V * 64 * WPG.
// Gate kernels exist for 2, 4 and 8 wavefronts per slot (a tuning choice);
// the codec and readout kernels use 2.
template <int SRC, int DST, bool GATE>
static hipError_t launch_job(const GateDesc &gd, const DevPtrs &P, const IOPtrs &io, int grid, hipStream_t st,
                             int wpg = 2, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr)
{
    const int threads = 64 * wpg;
    if (P.C % threads) return hipErrorInvalidValue;
    const int V = P.C / threads;
    if (gd.entropy) {   // the entropy stage: 2048-double chunks, two wavefronts per chunk
        if (V != 16 || wpg != 2) return hipErrorInvalidValue;
        launch_vw<16, 2, SRC, DST, GATE, true>(gd, P, io, grid, st, t0, t1);
        return hipGetLastError();
    }
    const int key = wpg * 100 + V;
    switch (key) {
    case 201: launch_vw<1, 2, SRC, DST, GATE>(gd, P, io, grid, st, t0, t1); break;
    case 202: launch_vw<2, 2, SRC, DST, GATE>(gd, P, io, grid, st, t0, t1); break;
    case 204: launch_vw<4, 2, SRC, DST, GATE>(gd, P, io, grid, st, t0, t1); break;
    case 208: launch_vw<8, 2, SRC, DST, GATE>(gd, P, io, grid, st, t0, t1); break;
    case 216: launch_vw<16, 2, SRC, DST, GATE>(gd, P, io, grid, st, t0, t1); break;
    default:
        if (!GATE) return hipErrorInvalidValue;
        switch (key) {
        case 401: launch_vw<1, 4, SRC, DST, GATE>(gd, P, io, grid, st, t0, t1); break;
        case 402: launch_vw<2, 4, SRC, DST, GATE>(gd, P, io, grid, st, t0, t1); break;
        case 404: launch_vw<4, 4, SRC, DST, GATE>(gd, P, io, grid, st, t0, t1); break;
        case 408: launch_vw<8, 4, SRC, DST, GATE>(gd, P, io, grid, st, t0, t1); break;
        case 801: launch_vw<1, 8, SRC, DST, GATE>(gd, P, io, grid, st, t0, t1); break;
        case 802: launch_vw<2, 8, SRC, DST, GATE>(gd, P, io, grid, st, t0, t1); break;
        case 804: launch_vw<4, 8, SRC, DST, GATE>(gd, P, io, grid, st, t0, t1); break;
        default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

hipError_t launch_gate(const GateDesc &gd, const DevPtrs &P, int grid, hipStream_t st, int wpg, hipEvent_t t0,
                       hipEvent_t t1)
{
    IOPtrs io = {};
    return launch_job<SRC_ARENA, DST_ARENA, true>(gd, P, io, grid, st, wpg, t0, t1);
}

template <int V>
static void launch_list_v(const GateDesc &gd, const DevPtrs &P, const IOPtrs &io, int list, int grid, hipStream_t st)
{
    if (list == 1)
        hipLaunchKernelGGL((job_kernel<V, 2, SRC_ARENA, DST_ARENA, true, 1>), dim3(grid), dim3(256), 0, st, gd, P, io);
    else
        hipLaunchKernelGGL((job_kernel<V, 2, SRC_ARENA, DST_ARENA, true, 2>), dim3(grid), dim3(256), 0, st, gd, P, io);
}

template <int V, bool ENT = false>
static void launch_run_v(const GateDesc &gd, const DevPtrs &P, const IOPtrs &io, int grid, hipStream_t st,
                         hipEvent_t t0, hipEvent_t t1)
{
    if (t0)
        hipExtLaunchKernelGGL((job_kernel<V, 2, SRC_ARENA, DST_ARENA, true, 3, ENT>), dim3(grid), dim3(256), 0, st, t0,
                              t1, 0, gd, P, io);
    else
        hipLaunchKernelGGL((job_kernel<V, 2, SRC_ARENA, DST_ARENA, true, 3, ENT>), dim3(grid), dim3(256), 0, st, gd, P,
                           io);
}

hipError_t launch_gate_run(const GateDesc &gd, const DevPtrs &P, const GateDesc *run, int nrun, int grid,
                           hipStream_t st, hipEvent_t t0, hipEvent_t t1)
{
    if (nrun < 1 || nrun > kMaxRun || grid < 1 || P.C % 128) return hipErrorInvalidValue;
    IOPtrs io = {};
    io.run = run;
    io.nrun = nrun;
    if (gd.entropy) {
        if (P.C != kCMax) return hipErrorInvalidValue;
        launch_run_v<16, true>(gd, P, io, grid, st, t0, t1);
        return hipGetLastError();
    }
    switch (P.C / 128) {
    case 1: launch_run_v<1>(gd, P, io, grid, st, t0, t1); break;
    case 2: launch_run_v<2>(gd, P, io, grid, st, t0, t1); break;
    case 4: launch_run_v<4>(gd, P, io, grid, st, t0, t1); break;
    case 8: launch_run_v<8>(gd, P, io, grid, st, t0, t1); break;
    case 16: launch_run_v<16>(gd, P, io, grid, st, t0, t1); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_group_run(const GateDesc &gd, const DevPtrs &P, const GateDesc *run, int nrun, int grid,
                            hipStream_t st, hipEvent_t t0, hipEvent_t t1)
{
    if (nrun < 1 || nrun > kMaxRun || grid < 1 || P.C != kCMax || gd.job_type != J_GROUP || gd.entropy)
        return hipErrorInvalidValue;
    IOPtrs io = {};
    io.run = run;
    io.nrun = nrun;
    // two chunk-index bits: 256 threads, two workgroups per CU; three: 512, one
    if (gd.pair_bit3) {
        if (t0)
            hipExtLaunchKernelGGL((group_kernel<16, 3>), dim3(grid), dim3(512), 0, st, t0, t1, 0, gd, P, io);
        else
            hipLaunchKernelGGL((group_kernel<16, 3>), dim3(grid), dim3(512), 0, st, gd, P, io);
    } else {
        if (t0)
            hipExtLaunchKernelGGL((group_kernel<16, 2>), dim3(grid), dim3(256), 0, st, t0, t1, 0, gd, P, io);
        else
            hipLaunchKernelGGL((group_kernel<16, 2>), dim3(grid), dim3(256), 0, st, gd, P, io);
    }
    return hipGetLastError();
}

hipError_t launch_gate_list(const GateDesc &gd, const DevPtrs &P, const CachePtrs &cp, int list, int grid,
                            hipStream_t st)
{
    if ((list != 1 && list != 2) || grid < 1 || grid > kMaxGrid / 2 || P.C % 128 || gd.entropy)
        return hipErrorInvalidValue;
    IOPtrs io = {};
    io.role = cp.role;
    io.owner = cp.owner;
    io.cparts = cp.parts;
    switch (P.C / 128) {
    case 1: launch_list_v<1>(gd, P, io, list, grid, st); break;
    case 2: launch_list_v<2>(gd, P, io, list, grid, st); break;
    case 4: launch_list_v<4>(gd, P, io, list, grid, st); break;
    case 8: launch_list_v<8>(gd, P, io, list, grid, st); break;
    case 16: launch_list_v<16>(gd, P, io, list, grid, st); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_cache_copy(const GateDesc &gd, const DevPtrs &P, const CachePtrs &cp, hipStream_t st)
{
    hipLaunchKernelGGL(cache_copy_kernel, dim3(kCopyGrid), dim3(kWG), 0, st, gd, P, cp, cp.parts);
    return hipGetLastError();
}

hipError_t launch_cache_plan(const GateDesc &gd, const DevPtrs &P, const CachePtrs &cp, hipStream_t st)
{
    const uint64_t jobs = job_stop(gd) - job_begin(gd);
    if (cp.tsize < 2 * jobs || (cp.tsize & (cp.tsize - 1))) return hipErrorInvalidValue;
    const uint64_t hb = std::max<uint64_t>(1, std::min<uint64_t>((jobs + kWG / 64 - 1) / (kWG / 64), 65535));
    hipLaunchKernelGGL(cache_hash_kernel, dim3((unsigned)hb), dim3(kWG), 0, st, gd, P, cp);
    const uint64_t db = (jobs + kWG - 1) / kWG;
    if (db > 0x7FFFFFFFull) return hipErrorInvalidValue;
    hipLaunchKernelGGL(cache_dedupe_kernel, dim3((unsigned)std::max<uint64_t>(1, db)), dim3(kWG), 0, st, gd, cp);
    return hipGetLastError();
}

hipError_t launch_permute(const GateDesc &gd, const DevPtrs &P, int grid, hipStream_t st)
{
    hipLaunchKernelGGL(permute_kernel, dim3(grid), dim3(kWG), 0, st, gd, P);
    return hipGetLastError();
}

hipError_t launch_rollback(const GateDesc &gd, const DevPtrs &P, int grid, hipStream_t st)
{
    hipLaunchKernelGGL(rollback_kernel, dim3(grid), dim3(kWG), 0, st, gd, P);
    return hipGetLastError();
}

hipError_t launch_encode_raw(const GateDesc &gd, const DevPtrs &P, const IOPtrs &io, int grid, hipStream_t st)
{
    return launch_job<SRC_RAW, DST_SLOTS, false>(gd, P, io, grid, st);
}

hipError_t launch_decode_slots(const GateDesc &gd, const DevPtrs &P, const IOPtrs &io, int grid, hipStream_t st)
{
    return launch_job<SRC_SLOTS, DST_RAW, false>(gd, P, io, grid, st);
}

hipError_t launch_readout(const GateDesc &gd, const DevPtrs &P, const IOPtrs &io, int grid, hipStream_t st)
{
    return launch_job<SRC_ARENA, DST_RAW, false>(gd, P, io, grid, st);
}

hipError_t launch_moments(const GateDesc &gd, const DevPtrs &P, const IOPtrs &io, int grid, hipStream_t st)
{
    return launch_job<SRC_ARENA, DST_MOMENTS, false>(gd, P, io, grid, st);
}

hipError_t launch_chunk_stats(const GateDesc &gd, const DevPtrs &P, const IOPtrs &io, int grid, hipStream_t st)
{
    return launch_job<SRC_ARENA, DST_CSTATS, false>(gd, P, io, grid, st);
}

hipError_t launch_level_sizes(const GateDesc &gd, const DevPtrs &P, const IOPtrs &io, int grid, hipStream_t st)
{
    return launch_job<SRC_ARENA, DST_LSIZES, false>(gd, P, io, grid, st);
}

// partial sums of conj(a) . b over interleaved complex values, one pair per workgroup
__global__ __launch_bounds__(kWG) void dot_kernel(const double *a, const double *b, uint64_t npairs, double *partials)
{
    __shared__ double red[kWG / 64][2];
    double re = 0.0, im = 0.0;
    for (uint64_t i = (uint64_t)blockIdx.x * kWG + threadIdx.x; i < npairs; i += (uint64_t)gridDim.x * kWG) {
        const double ar = a[2 * i], ai = a[2 * i + 1], br = b[2 * i], bi = b[2 * i + 1];
        re += ar * br + ai * bi;
        im += ar * bi - ai * br;
    }
    for (int d = 32; d >= 1; d >>= 1) {
        re += __shfl_down(re, d, 64);
        im += __shfl_down(im, d, 64);
    }
    if ((threadIdx.x & 63) == 0) { red[threadIdx.x >> 6][0] = re; red[threadIdx.x >> 6][1] = im; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = 0.0, m = 0.0;
        for (int w = 0; w < kWG / 64; ++w) { r += red[w][0]; m += red[w][1]; }
        partials[2 * blockIdx.x] = r;
        partials[2 * blockIdx.x + 1] = m;
    }
}

hipError_t launch_dot(const double *a, const double *b, uint64_t npairs, double *partials, int grid, hipStream_t st)
{
    hipLaunchKernelGGL(dot_kernel, dim3(grid), dim3(kWG), 0, st, a, b, npairs, partials);
    return hipGetLastError();
}

__global__ __launch_bounds__(kWG) void zero_u64_kernel(uint64_t *p, uint64_t n)
{
    for (uint64_t i = (uint64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kWG) p[i] = 0ull;
}

hipError_t launch_zero_u64(uint64_t *p, uint64_t n, hipStream_t st)
{
    const uint64_t blocks = (n + kWG - 1) / kWG;
    const int grid = (int)(blocks < 4096 ? (blocks ? blocks : 1) : 4096);
    hipLaunchKernelGGL(zero_u64_kernel, dim3(grid), dim3(kWG), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_fill_table(const DevPtrs &P, uint64_t entry0, uint64_t entry_rest, hipStream_t st)
{
    uint64_t blocks = (P.nchunks + kWG - 1) / kWG;
    int grid = (int)(blocks < 65536 ? blocks : 65536);
    hipLaunchKernelGGL(fill_table_kernel, dim3(grid), dim3(kWG), 0, st, P.table, P.nchunks, entry0, entry_rest);
    return hipGetLastError();
}

hipError_t launch_compact(const DevPtrs &P, uint32_t *dst_arena, uint64_t *scratch, uint64_t *block_sums,
                          uint64_t nblocks_scan, hipStream_t st)
{
    hipLaunchKernelGGL(scan_local_kernel, dim3((unsigned)nblocks_scan), dim3(kWG), 0, st, P.table, P.nchunks, scratch,
                       block_sums);
    hipLaunchKernelGGL(scan_blocks_kernel, dim3(1), dim3(kWG), 0, st, block_sums, nblocks_scan);
    uint64_t waves = P.nchunks;
    uint64_t blocks = (waves * 64 + kWG - 1) / kWG;
    int grid = (int)(blocks < 8192 ? blocks : 8192);
    hipLaunchKernelGGL(compact_copy_kernel, dim3(grid), dim3(kWG), 0, st, P, dst_arena, scratch, block_sums);
    return hipGetLastError();
}

}  // namespace qcz

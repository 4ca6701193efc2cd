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

namespace qcz {

// Sig_Bit_Count of Eq. (12) for binary64 (12 sign/exponent bits minus the
// exponent of the bound) per level: lossless, 1e-5, 1e-4, 1e-3, 1e-2, 1e-1.
__constant__ int kSig[kLevels] = {64, 29, 26, 22, 19, 16};

enum { SRC_ARENA = 0, SRC_RAW = 1, SRC_SLOTS = 2 };
enum { DST_ARENA = 0, DST_RAW = 1, DST_SLOTS = 2, DST_MOMENTS = 3 };

// ---------------------------------------------------------------------------
// bit helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t d2u(double x) { return (uint64_t)__double_as_longlong(x); }
__device__ __forceinline__ double u2d(uint64_t b) { return __longlong_as_double((long long)b); }

__device__ __forceinline__ uint64_t trunc_bits(uint64_t b, int K)
{
    return K >= 64 ? b : (b & ~((1ull << (64 - K)) - 1ull));
}

// identical leading bytes of two values, most significant first, capped at 3
__device__ __forceinline__ int lead_bytes(uint64_t cur, uint64_t prev)
{
    uint64_t d = cur ^ prev;
    if (d == 0) return 3;
    int L = __clzll((long long)d) >> 3;
    return L < 3 ? L : 3;
}

__device__ __forceinline__ int resid_bits(int K, int L)
{
    int r = K - 8 * L;
    return r > 0 ? r : 0;
}

__device__ __forceinline__ uint64_t top_mask(int nbits)  // 0 <= nbits <= 24
{
    return nbits <= 0 ? 0ull : (~0ull << (64 - nbits));
}

__device__ __forceinline__ bool subnormal(uint64_t b)
{
    return ((b >> 52) & 0x7FFull) == 0 && (b & 0xFFFFFFFFFFFFFull) != 0;
}

__device__ __forceinline__ int clampw(int i) { return i < kBufWords - 1 ? i : kBufWords - 1; }

// r bits (r <= 64) at bit offset o of the word stream starting at b[base]
__device__ __forceinline__ uint64_t read_bits(const uint32_t *b, int base, uint32_t o, int r)
{
    if (r == 0) return 0;
    int wi = base + (int)(o >> 5);
    int sh = (int)(o & 31);
    uint64_t w0 = b[clampw(wi)], w1 = b[clampw(wi + 1)], w2 = b[clampw(wi + 2)];
    uint64_t v = (w0 | (w1 << 32)) >> sh;
    if (sh) v |= w2 << (64 - sh);
    return r >= 64 ? v : (v & ((1ull << r) - 1ull));
}

// ---------------------------------------------------------------------------
// group scans: a group is the 128 threads (two wavefronts) of one chunk slot
// ---------------------------------------------------------------------------
__device__ __forceinline__ void wave_scan3(uint32_t &a, uint32_t &b, uint32_t &c)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t ya = __shfl_up(a, d, 64), yb = __shfl_up(b, d, 64), yc = __shfl_up(c, d, 64);
        if (lane >= d) { a += ya; b += yb; c += yc; }
    }
}

// exclusive sums of (v0, v1, v2) over the group; totals in tot
__device__ void group_scan3(uint32_t v0, uint32_t v1, uint32_t v2, uint32_t *sh, uint32_t ex[3], uint32_t tot[3])
{
    uint32_t a = v0, b = v1, c = v2;
    wave_scan3(a, b, c);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 63) { sh[4 * w] = a; sh[4 * w + 1] = b; sh[4 * w + 2] = c; }
    __syncthreads();
    const int w0 = w & ~1;
    const bool odd = (w & 1) != 0;
    uint32_t p0 = sh[4 * w0], p1 = sh[4 * w0 + 1], p2 = sh[4 * w0 + 2];
    uint32_t q0 = sh[4 * w0 + 4], q1 = sh[4 * w0 + 5], q2 = sh[4 * w0 + 6];
    ex[0] = (odd ? p0 : 0) + a - v0;
    ex[1] = (odd ? p1 : 0) + b - v1;
    ex[2] = (odd ? p2 : 0) + c - v2;
    tot[0] = p0 + q0;
    tot[1] = p1 + q1;
    tot[2] = p2 + q2;
    __syncthreads();
}

// "last writer" combine of per-byte carries: bits 24..26 flag bytes 0..2,
// bits 8j..8j+7 hold byte j; the later operand wins where it is defined.
__device__ __forceinline__ uint32_t carry_op(uint32_t a, uint32_t b)
{
    uint32_t bm = (b >> 24) & 7u;
    uint32_t sel = ((bm & 1u) ? 0xFFu : 0u) | ((bm & 2u) ? 0xFF00u : 0u) | ((bm & 4u) ? 0xFF0000u : 0u);
    return ((a | b) & 0x07000000u) | (b & sel) | (a & ~sel & 0xFFFFFFu);
}

// exclusive carry scan over the group (identity 0)
__device__ uint32_t group_scan_carry(uint32_t v, uint32_t *sh)
{
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t y = __shfl_up(x, d, 64);
        if (lane >= d) x = carry_op(y, x);
    }
    uint32_t e = __shfl_up(x, 1, 64);
    if (lane == 0) e = 0;
    if (lane == 63) sh[4 * w + 3] = x;
    __syncthreads();
    if (w & 1) e = carry_op(sh[4 * (w - 1) + 3], e);
    __syncthreads();
    return e;
}

// exclusive "last value with flag" scan over the group
__device__ void group_scan_last(bool has, uint64_t val, uint32_t *sh, bool &ehas, uint64_t &eval)
{
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint32_t h = has ? 1u : 0u, lo = (uint32_t)val, hi = (uint32_t)(val >> 32);
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t yh = __shfl_up(h, d, 64), ylo = __shfl_up(lo, d, 64), yhi = __shfl_up(hi, d, 64);
        if (lane >= d && !h) { h = yh; lo = ylo; hi = yhi; }
    }
    uint32_t eh = __shfl_up(h, 1, 64), elo = __shfl_up(lo, 1, 64), ehi = __shfl_up(hi, 1, 64);
    if (lane == 0) eh = 0;
    if (lane == 63) { sh[16 + 4 * w] = h; sh[16 + 4 * w + 1] = lo; sh[16 + 4 * w + 2] = hi; }
    __syncthreads();
    if ((w & 1) && !eh) {
        eh = sh[16 + 4 * (w - 1)];
        elo = sh[16 + 4 * (w - 1) + 1];
        ehi = sh[16 + 4 * (w - 1) + 2];
    }
    __syncthreads();
    ehas = eh != 0;
    eval = ((uint64_t)ehi << 32) | elo;
}

// ---------------------------------------------------------------------------
// decode: the chunk staged in b[] -> the V values this thread owns
// ---------------------------------------------------------------------------
template <int V>
__device__ void decode_group(const uint32_t *b, bool active, int C, int lt, uint32_t *sh, uint64_t (&t)[V])
{
    const uint32_t hdr = active ? b[0] : (uint32_t)M_CONST2;
    const int mode = (int)(hdr & 3u);
    int lev = (int)((hdr >> 2) & 7u);
    if (lev >= kLevels) lev = 0;
    const int K = kSig[lev];
    const int first = lt * V;
    const uint32_t vmask = (V >= 32) ? 0xFFFFFFFFu : ((1u << V) - 1u);
    uint32_t stored = 0;
    if (mode == M_PACK) stored = vmask;
    else if (mode == M_SPARSE) stored = (b[clampw(1 + (first >> 5))] >> (first & 31)) & vmask;
    const uint32_t cnt = __popc(stored);

    uint32_t ex[3], tot[3];
    group_scan3(cnt, 0, 0, sh, ex, tot);
    const uint32_t rank0 = ex[0], nnz = tot[0];
    const int codes_w0 = (mode == M_SPARSE) ? 1 + ((C + 31) >> 5) : 1;
    const int res_w0 = codes_w0 + (int)((nnz + 15) >> 4);

    uint64_t cw = 0;
    if (cnt) {
        uint32_t bit = 2 * rank0;
        int wi = codes_w0 + (int)(bit >> 5);
        uint64_t lo = b[clampw(wi)], hi = b[clampw(wi + 1)];
        cw = ((hi << 32) | lo) >> (bit & 31);
    }
    int Lk[V];
    uint32_t rsum = 0;
#pragma unroll
    for (int k = 0; k < V; ++k) {
        uint32_t lr = __popc(stored & ((1u << k) - 1u));
        Lk[k] = (int)((cw >> (2 * lr)) & 3u);
        if ((stored >> k) & 1u) rsum += (uint32_t)resid_bits(K, Lk[k]);
    }
    group_scan3(rsum, 0, 0, sh, ex, tot);
    uint32_t o = ex[0];

    uint32_t carry = 0;
#pragma unroll
    for (int k = 0; k < V; ++k) {
        uint64_t p = 0;
        if ((stored >> k) & 1u) {
            int r = resid_bits(K, Lk[k]);
            uint64_t R = read_bits(b, res_w0, o, r);
            o += (uint32_t)r;
            p = (K >= 64) ? R : (R << (64 - K));
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                if (Lk[k] <= j) {
                    carry = (carry & ~(0xFFu << (8 * j))) | ((uint32_t)((p >> (56 - 8 * j)) & 0xFFu) << (8 * j));
                    carry |= 1u << (24 + j);
                }
            }
        }
        t[k] = p;
    }
    uint32_t inc = carry_op(0x07000000u, group_scan_carry(carry, sh));
    uint64_t prev = ((uint64_t)(inc & 0xFFu) << 56) | ((uint64_t)((inc >> 8) & 0xFFu) << 48) |
                    ((uint64_t)((inc >> 16) & 0xFFu) << 40);
    if (mode == M_CONST2) {
        uint64_t t0 = active ? ((uint64_t)b[1] | ((uint64_t)b[2] << 32)) : 0ull;
        uint64_t t1 = active ? ((uint64_t)b[3] | ((uint64_t)b[4] << 32)) : 0ull;
#pragma unroll
        for (int k = 0; k < V; ++k) t[k] = ((first + k) & 1) ? t1 : t0;
    } else {
#pragma unroll
        for (int k = 0; k < V; ++k) {
            if ((stored >> k) & 1u) {
                uint64_t v = (prev & top_mask(8 * Lk[k])) | t[k];
                t[k] = v;
                prev = v;
            } else {
                t[k] = 0;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// encode
// ---------------------------------------------------------------------------
template <int V>
struct EncPlan {
    uint64_t t[V];      // truncated values
    uint32_t codes;     // PACK codes of my positions (2 bits each)
    uint32_t scodes;    // SPARSE codes of my nonzero positions, in rank order
    uint32_t nzm;       // my nonzero positions
    uint32_t pack_off;  // bit offset of my PACK residuals
    uint32_t sp_off;    // bit offset of my SPARSE residuals
    uint32_t rank0;     // rank of my first nonzero
    uint32_t nnz;
    uint64_t c0, c1;    // CONST2 values (truncated values 0 and 1)
    int mode, lev, K;
    uint32_t size;
};

template <int V>
__device__ void encode_plan(const uint64_t (&x)[V], uint64_t xprev, uint64_t x0, uint64_t x1, int lev_req,
                            bool active, int C, int lt, uint32_t *sh, EncPlan<V> &e)
{
    const int first = lt * V;
    uint32_t sub = 0;
#pragma unroll
    for (int k = 0; k < V; ++k) sub |= (active && subnormal(x[k])) ? 1u : 0u;
    uint32_t ex[3], tot[3];
    group_scan3(sub, 0, 0, sh, ex, tot);
    const int lev = (tot[0] != 0) ? 0 : lev_req;       // a chunk with a subnormal is kept lossless
    const int K = kSig[lev];
    const uint64_t tp = trunc_bits(xprev, K), t0 = trunc_bits(x0, K), t1 = trunc_bits(x1, K);

    uint32_t bad2 = 0, rp = 0, nzm = 0, codes = 0;
    uint64_t prev = tp, lastnz = 0;
#pragma unroll
    for (int k = 0; k < V; ++k) {
        uint64_t tk = active ? trunc_bits(x[k], K) : 0ull;
        e.t[k] = tk;
        bad2 += (tk != (((first + k) & 1) ? t1 : t0)) ? 1u : 0u;
        int L = lead_bytes(tk, prev);
        codes |= (uint32_t)L << (2 * k);
        rp += (uint32_t)resid_bits(K, L);
        prev = tk;
        if (tk != 0) { nzm |= 1u << k; lastnz = tk; }
    }
    const uint32_t cnt = __popc(nzm);
    group_scan3(bad2, rp, cnt, sh, ex, tot);
    const bool const2 = tot[0] == 0;
    const uint32_t RP = tot[1], NNZ = tot[2];
    e.pack_off = ex[1];
    e.rank0 = ex[2];
    e.nnz = NNZ;
    bool ph;
    uint64_t pv;
    group_scan_last(cnt != 0, lastnz, sh, ph, pv);
    uint64_t sprev = ph ? pv : 0ull;
    uint32_t rs = 0, scodes = 0, j = 0;
#pragma unroll
    for (int k = 0; k < V; ++k) {
        if ((nzm >> k) & 1u) {
            int L = lead_bytes(e.t[k], sprev);
            scodes |= (uint32_t)L << (2 * j);
            ++j;
            rs += (uint32_t)resid_bits(K, L);
            sprev = e.t[k];
        }
    }
    group_scan3(rs, 0, 0, sh, ex, tot);
    e.sp_off = ex[0];
    const uint32_t RS = tot[0];
    const uint32_t pack_size = 4u + 4u * (uint32_t)((C + 15) / 16) + (RP + 7u) / 8u;
    const uint32_t sparse_size = 4u + 4u * (uint32_t)((C + 31) / 32) + 4u * ((NNZ + 15u) / 16u) + (RS + 7u) / 8u;
    e.c0 = t0;
    e.c1 = t1;
    e.codes = codes;
    e.scodes = scodes;
    e.nzm = nzm;
    e.lev = lev;
    e.K = K;
    if (const2) { e.mode = M_CONST2; e.size = 20; }
    else if (sparse_size < pack_size) { e.mode = M_SPARSE; e.size = sparse_size; }
    else { e.mode = M_PACK; e.size = pack_size; }
}

// Bit writer into LDS words: the first and the last word a thread touches
// may be shared with its neighbours (atomic OR); words in between are its own.
struct BitOut {
    uint32_t *w;
    int wi;
    int nb;
    uint64_t acc;
    bool first;
    __device__ void init(uint32_t *base, uint32_t bitoff) { w = base; wi = (int)(bitoff >> 5); nb = (int)(bitoff & 31); acc = 0; first = true; }
    __device__ __forceinline__ void put32(uint64_t v, int n)  // n <= 32, nb < 32 on entry
    {
        if (n == 0) return;
        acc |= v << nb;
        nb += n;
        if (nb >= 32) {
            int idx = clampw(wi);
            if (first) atomicOr(&w[idx], (uint32_t)acc);
            else w[idx] = (uint32_t)acc;
            first = false;
            ++wi;
            acc >>= 32;
            nb -= 32;
        }
    }
    __device__ __forceinline__ void put(uint64_t v, int n)
    {
        if (n > 32) { put32(v & 0xFFFFFFFFull, 32); put32(v >> 32, n - 32); }
        else put32(v, n);
    }
    __device__ __forceinline__ void flush()
    {
        if (nb > 0) atomicOr(&w[clampw(wi)], (uint32_t)acc);
    }
};

__device__ __forceinline__ uint64_t residual_of(uint64_t t, int K, int r)
{
    uint64_t sig = (K >= 64) ? t : (t >> (64 - K));
    return r >= 64 ? sig : (sig & ((1ull << r) - 1ull));
}

// write the planned stream into b[] (already zeroed); no barriers inside
template <int V>
__device__ void encode_emit(uint32_t *b, const EncPlan<V> &e, int C, int lt)
{
    const int first = lt * V;
    if (lt == 0) b[0] = (uint32_t)e.mode | ((uint32_t)e.lev << 2);
    if (e.mode == M_CONST2) {
        if (lt == 0) {
            b[1] = (uint32_t)e.c0; b[2] = (uint32_t)(e.c0 >> 32);
            b[3] = (uint32_t)e.c1; b[4] = (uint32_t)(e.c1 >> 32);
        }
        return;
    }
    const int K = e.K;
    if (e.mode == M_PACK) {
        const uint32_t bit = 2u * (uint32_t)first;
        if (V == 16) b[1 + (bit >> 5)] = e.codes;
        else atomicOr(&b[1 + (bit >> 5)], e.codes << (bit & 31));
        BitOut bo;
        bo.init(b + 1 + C / 16, e.pack_off);
#pragma unroll
        for (int k = 0; k < V; ++k) {
            int L = (int)((e.codes >> (2 * k)) & 3u);
            int r = resid_bits(K, L);
            bo.put(residual_of(e.t[k], K, r), r);
        }
        bo.flush();
    } else {  // M_SPARSE
        if (e.nzm) atomicOr(&b[1 + (first >> 5)], e.nzm << (first & 31));
        const int codes_w0 = 1 + ((C + 31) >> 5);
        const uint32_t cnt = __popc(e.nzm);
        if (cnt) {
            uint32_t bit = 2u * e.rank0;
            uint64_t v = (uint64_t)e.scodes << (bit & 31);
            int wi = codes_w0 + (int)(bit >> 5);
            if ((uint32_t)v) atomicOr(&b[clampw(wi)], (uint32_t)v);
            if ((uint32_t)(v >> 32)) atomicOr(&b[clampw(wi + 1)], (uint32_t)(v >> 32));
        }
        BitOut bo;
        bo.init(b + codes_w0 + (int)((e.nnz + 15u) >> 4), e.sp_off);
        uint32_t j = 0;
#pragma unroll
        for (int k = 0; k < V; ++k) {
            if ((e.nzm >> k) & 1u) {
                int L = (int)((e.scodes >> (2 * j)) & 3u);
                ++j;
                int r = resid_bits(K, L);
                bo.put(residual_of(e.t[k], K, r), r);
            }
        }
        bo.flush();
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

// a diagonal gate leaves chunk c alone when every phase reachable in it is 1
__device__ bool diag_touches(const GateDesc &gd, uint64_t c, int cb)
{
    const int nidx = gd.kind == K_DIAG1 ? 2 : 4;
    for (int idx = 0; idx < nidx; ++idx) {
        int b1 = idx & 1, b2 = idx >> 1;
        if (gd.q >= cb && (int)((c >> (gd.q - cb)) & 1ull) != b1) continue;
        if (gd.kind == K_DIAG2 && gd.q2 >= cb && (int)((c >> (gd.q2 - cb)) & 1ull) != b2) continue;
        if (!unit_phase(gd.m[2 * idx], gd.m[2 * idx + 1])) return true;
    }
    return false;
}

__device__ __forceinline__ uint64_t deposit(const GateDesc &gd, uint64_t k)
{
    uint64_t c = gd.fixed_val;
    for (int bpos = 0; bpos < gd.nchunk_bits; ++bpos) {
        if (!((gd.fixed_mask >> bpos) & 1ull)) {
            c |= (k & 1ull) << bpos;
            k >>= 1;
        }
    }
    return c;
}

// chunk id of enumerated position `item`
__device__ __forceinline__ uint64_t item_chunk(const GateDesc &gd, uint64_t item)
{
    if (gd.job_type == J_PAIR) {
        uint64_t c = deposit(gd, item >> 1);
        return (item & 1ull) ? (c | gd.pair_bit) : c;
    }
    return deposit(gd, item);
}

__device__ void apply_gate(const GateDesc &gd, double *v0, double *v1, uint64_t c0, uint64_t c1, bool a0, bool a1,
                           int cb)
{
    const int tid = threadIdx.x;
    const int ca = 1 << cb;
    const uint64_t cm = gd.cm;
    const double *m = gd.m;
    if (gd.job_type == J_PAIR) {
        if (!(a0 && a1)) return;
        for (int k = tid; k < ca; k += kWG) {
            uint64_t i = (c0 << cb) | (uint64_t)k;
            if ((i & cm) != cm) continue;
            double ar = v0[2 * k], ai = v0[2 * k + 1], br = v1[2 * k], bi = v1[2 * k + 1];
            if (gd.kind == K_X) {
                v0[2 * k] = br; v0[2 * k + 1] = bi; v1[2 * k] = ar; v1[2 * k + 1] = ai;
            } else {
                double yr, yi, zr, zi;
                lin2(m[0], m[1], m[2], m[3], ar, ai, br, bi, yr, yi);
                lin2(m[4], m[5], m[6], m[7], ar, ai, br, bi, zr, zi);
                v0[2 * k] = yr; v0[2 * k + 1] = yi; v1[2 * k] = zr; v1[2 * k + 1] = zi;
            }
        }
        return;
    }
    const bool pairwise = gd.kind == K_U1 || gd.kind == K_X;
    const int units = pairwise ? ca / 2 : ca;
    for (int w = tid; w < 2 * units; w += kWG) {
        const int s = w >= units ? 1 : 0;
        const int u = w - s * units;
        if (!(s ? a1 : a0)) continue;
        double *v = s ? v1 : v0;
        const uint64_t base = (s ? c1 : c0) << cb;
        if (pairwise) {
            const int q = gd.q;
            const int k0 = ((u >> q) << (q + 1)) | (u & ((1 << q) - 1));
            const int k1 = k0 | (1 << q);
            const uint64_t i = base | (uint64_t)k0;
            if ((i & cm) != cm) continue;
            double ar = v[2 * k0], ai = v[2 * k0 + 1], br = v[2 * k1], bi = v[2 * k1 + 1];
            if (gd.kind == K_X) {
                v[2 * k0] = br; v[2 * k0 + 1] = bi; v[2 * k1] = ar; v[2 * k1 + 1] = ai;
            } else {
                double yr, yi, zr, zi;
                lin2(m[0], m[1], m[2], m[3], ar, ai, br, bi, yr, yi);
                lin2(m[4], m[5], m[6], m[7], ar, ai, br, bi, zr, zi);
                v[2 * k0] = yr; v[2 * k0 + 1] = yi; v[2 * k1] = zr; v[2 * k1 + 1] = zi;
            }
        } else {
            const uint64_t i = base | (uint64_t)u;
            if ((i & cm) != cm) continue;
            if (gd.kind == K_MCZ) {
                v[2 * u] = -v[2 * u];
                v[2 * u + 1] = -v[2 * u + 1];
            } else {
                int idx = (int)((i >> gd.q) & 1ull);
                if (gd.kind == K_DIAG2) idx += 2 * (int)((i >> gd.q2) & 1ull);
                double yr, yi;
                dmul(m[2 * idx], m[2 * idx + 1], v[2 * u], v[2 * u + 1], yr, yi);
                v[2 * u] = yr; v[2 * u + 1] = yi;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// the job kernel
// ---------------------------------------------------------------------------
template <int V, int SRC, int DST, bool GATE>
__global__ __launch_bounds__(kWG) void job_kernel(GateDesc gd, DevPtrs P, IOPtrs io)
{
    __shared__ uint32_t buf[2][kBufWords];
    __shared__ uint32_t sh[32];
    __shared__ uint64_t sh_off[2];
    __shared__ int sh_ok[2];
    __shared__ int sh_src_ok[2];
    __shared__ uint64_t sh_acc[4];
    __shared__ double sh_mom[kWG / 64][4];

    DevState *ds = P.ds;
    if (DST == DST_ARENA && ds->stop) return;

    const int tid = threadIdx.x, s = tid >> 7, lt = tid & (kGroup - 1);
    const int C = P.C;
    uint32_t *b = buf[s];
    double *vals = reinterpret_cast<double *>(b);
    const int first = lt * V;

    uint64_t acc_reenc = 0;
    int64_t acc_delta = 0;
    double mom_re = 0.0, mom_im = 0.0, mom_n2 = 0.0;

    for (uint64_t job = blockIdx.x; job < gd.njobs; job += gridDim.x) {
        const uint64_t item0 = 2 * job, item1 = 2 * job + 1;
        const bool valid0 = item0 < gd.nitems, valid1 = item1 < gd.nitems;
        uint64_t cc0 = 0, cc1 = 0;
        if (SRC == SRC_ARENA && !GATE && io.list) {
            cc0 = valid0 ? io.list[item0] : 0;
            cc1 = valid1 ? io.list[item1] : 0;
        } else {
            cc0 = valid0 ? item_chunk(gd, item0) + io.first : 0;
            cc1 = valid1 ? item_chunk(gd, item1) + io.first : 0;
        }
        bool act0 = valid0, act1 = valid1;
        if (GATE && gd.check_phase) {
            act0 = act0 && diag_touches(gd, cc0, P.cb);
            act1 = act1 && diag_touches(gd, cc1, P.cb);
        }
        const uint64_t item = s ? item1 : item0;
        const uint64_t c = s ? cc1 : cc0;
        const bool valid = s ? valid1 : valid0;
        const bool act = s ? act1 : act0;

        // 1. fetch
        uint64_t old_entry = 0;
        bool ok_src = true;
        if (SRC == SRC_ARENA) {
            if (valid) old_entry = P.table[c];
            const uint32_t size = (uint32_t)(old_entry & 0xFFFFull);
            const uint64_t off = old_entry >> 16;
            const uint32_t words = (size + 3u) >> 2;
            ok_src = words <= (uint32_t)(kBufWords - 8) && off + words <= P.arena_words && size >= 4;
            if (act && ok_src)
                for (uint32_t w = lt; w < words; w += kGroup) b[w] = P.arena[off + w];
            if (act && !ok_src && lt == 0 && ds) atomicExch(&ds->corrupt, 1);
        } else if (SRC == SRC_SLOTS) {
            const uint32_t size = valid ? io.sizes_in[item] : 0u;
            const uint32_t words = (size + 3u) >> 2;
            ok_src = words <= (uint32_t)(kBufWords - 8) && words <= io.slot_words && size >= 4;
            if (act && ok_src)
                for (uint32_t w = lt; w < words; w += kGroup) b[w] = io.slots_in[item * io.slot_words + w];
        } else {  // SRC_RAW
            if (act)
                for (int w = lt; w < C; w += kGroup) vals[w] = io.raw_in[item * (uint64_t)C + w];
        }
        if (lt == 0) sh_src_ok[s] = ok_src ? 1 : 0;
        __syncthreads();
        const bool src_ok0 = sh_src_ok[0] != 0, src_ok1 = sh_src_ok[1] != 0;

        // 2. decode
        if (SRC != SRC_RAW) {
            uint64_t t[V];
            decode_group<V>(b, act && ok_src, C, lt, sh, t);
            __syncthreads();
#pragma unroll
            for (int k = 0; k < V; ++k) vals[first + k] = u2d(t[k]);
            __syncthreads();
        }

        // 3. gate
        if (GATE) {
            apply_gate(gd, reinterpret_cast<double *>(buf[0]), reinterpret_cast<double *>(buf[1]), cc0, cc1,
                       act0 && src_ok0, act1 && src_ok1, P.cb);
            __syncthreads();
        }

        // 4. sink
        if (DST == DST_RAW) {
            if (act)
                for (int w = lt; w < C; w += kGroup) io.raw_out[item * (uint64_t)C + w] = vals[w];
        } else if (DST == DST_MOMENTS) {
            if (act) {
#pragma unroll
                for (int k = 0; k < V; k += 2) {
                    double re = vals[first + k], im = (k + 1 < V) ? vals[first + k + 1] : 0.0;
                    mom_re += re;
                    mom_im += im;
                    mom_n2 += re * re + im * im;
                }
                if (V == 1) {  // one value per thread: odd threads hold the imaginary parts
                    double v = vals[first];
                    mom_re -= (lt & 1) ? v : 0.0;
                    mom_im += (lt & 1) ? v : 0.0;
                    mom_n2 += 0.0;
                }
            }
        } else {
            // encode at the chunk's level
            uint64_t x[V];
#pragma unroll
            for (int k = 0; k < V; ++k) x[k] = d2u(vals[first + k]);
            const uint64_t xprev = lt ? d2u(vals[first - 1]) : 0ull;
            const uint64_t x0 = d2u(vals[0]), x1 = d2u(vals[1]);
            int lev_req;
            if (gd.fixed_level >= 0) lev_req = gd.fixed_level;
            else if (gd.per_block) lev_req = P.block_level[c >> gd.block_shift];
            else lev_req = ds->level;
            const bool enc = act && ok_src;
            EncPlan<V> e;
            encode_plan<V>(x, xprev, x0, x1, lev_req, enc, C, lt, sh, e);
            if (lt == 0) {
                uint64_t off = 0;
                int ok = 0;
                if (enc) {
                    if (DST == DST_ARENA) {
                        const uint64_t pad = (e.size + 3u) & ~3u;
                        off = atomicAdd((unsigned long long *)&ds->bump, (unsigned long long)pad);
                        ok = (off + pad <= ds->arena_cap) ? 1 : 0;
                        if (!ok) atomicExch(&ds->fail, 1);
                    } else {
                        ok = 1;
                    }
                }
                sh_off[s] = off;
                sh_ok[s] = ok;
            }
            __syncthreads();
            const uint32_t words = (e.size + 3u) >> 2;
            if (enc)
                for (uint32_t w = lt; w < words; w += kGroup) b[w] = 0u;
            __syncthreads();
            if (enc) encode_emit<V>(b, e, C, lt);
            __syncthreads();
            const int ok = sh_ok[s];
            if (ok) {
                if (DST == DST_ARENA) {
                    const uint64_t offw = sh_off[s] >> 2;
                    for (uint32_t w = lt; w < words; w += kGroup) P.arena[offw + w] = b[w];
                } else {
                    for (uint32_t w = lt; w < words; w += kGroup) io.slots_out[item * io.slot_words + w] = b[w];
                }
            }
            if (lt == 0 && valid) {
                if (DST == DST_ARENA) {
                    P.undo[item] = old_entry;
                    if (ok) {
                        P.table[c] = ((sh_off[s] >> 2) << 16) | (uint64_t)e.size;
                        const uint64_t old_pad = ((old_entry & 0xFFFFull) + 3ull) & ~3ull;
                        acc_delta += (int64_t)(((uint64_t)e.size + 3ull) & ~3ull) - (int64_t)old_pad;
                        acc_reenc += 1;
                    }
                } else {
                    io.sizes_out[item] = ok ? e.size : 0u;
                }
            }
        }
        __syncthreads();
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
        __syncthreads();
        if (tid == 0) {
            double A = 0, B = 0, Cc = 0;
            for (int w = 0; w < kWG / 64; ++w) { A += sh_mom[w][0]; B += sh_mom[w][1]; Cc += sh_mom[w][2]; }
            io.partials[4 * blockIdx.x] = A;
            io.partials[4 * blockIdx.x + 1] = B;
            io.partials[4 * blockIdx.x + 2] = Cc;
            io.partials[4 * blockIdx.x + 3] = 0.0;
        }
    }

    if (DST == DST_ARENA) {
        // per-workgroup totals, then the last workgroup closes the gate
        if (lt == 0) { sh_acc[2 * s] = (uint64_t)acc_delta; sh_acc[2 * s + 1] = acc_reenc; }
        __syncthreads();
        if (tid == 0) {
            const uint64_t d = sh_acc[0] + sh_acc[2];
            const uint64_t r = sh_acc[1] + sh_acc[3];
            if (d) atomicAdd((unsigned long long *)&ds->live, (unsigned long long)d);
            if (r) atomicAdd((unsigned long long *)&ds->reenc_cur, (unsigned long long)r);
            __threadfence();
            const uint32_t prev = atomicAdd(&ds->done, 1u);
            sh_ok[0] = (prev == gridDim.x - 1) ? 1 : 0;
        }
        __syncthreads();
        if (tid == 0 && sh_ok[0]) {
            __threadfence();
            const uint64_t live = atomicAdd((unsigned long long *)&ds->live, 0ull);
            const uint64_t bump = atomicAdd((unsigned long long *)&ds->bump, 0ull);
            const uint64_t reenc = atomicExch((unsigned long long *)&ds->reenc_cur, 0ull);
            GateLog lg;
            lg.live = live;
            lg.bump = bump;
            lg.reenc = reenc;
            lg.pad = 0;
            ds->log[gd.seq] = lg;
            const int fail = atomicExch(&ds->fail, 0);
            const int corrupt = atomicExch(&ds->corrupt, 0);
            int reason = STOP_NONE;
            if (corrupt) reason = STOP_CORRUPT;
            else if (fail) reason = STOP_ARENA;
            else if (ds->budget && live > ds->budget) reason = STOP_BUDGET;
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
        lg.live = atomicAdd((unsigned long long *)&ds->live, 0ull);
        lg.bump = atomicAdd((unsigned long long *)&ds->bump, 0ull);
        lg.reenc = 0;
        lg.pad = 0;
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
    for (uint64_t it = (uint64_t)blockIdx.x * kWG + threadIdx.x; it < gd.nitems; it += stride)
        P.table[item_chunk(gd, it)] = P.undo[it];
}

__global__ __launch_bounds__(kWG) void fill_table_kernel(uint64_t *table, uint64_t n, uint64_t e0, uint64_t erest)
{
    const uint64_t stride = (uint64_t)gridDim.x * kWG;
    for (uint64_t c = (uint64_t)blockIdx.x * kWG + threadIdx.x; c < n; c += stride) table[c] = c ? erest : e0;
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
        v[k] = c < n ? (((table[c] & 0xFFFFull) + 3ull) & ~3ull) : 0ull;
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
template <int SRC, int DST, bool GATE>
static hipError_t launch_job(const GateDesc &gd, const DevPtrs &P, const IOPtrs &io, int grid, hipStream_t st)
{
    const int V = P.C / kGroup;
    dim3 g(grid), blk(kWG);
    switch (V) {
    case 1: hipLaunchKernelGGL((job_kernel<1, SRC, DST, GATE>), g, blk, 0, st, gd, P, io); break;
    case 2: hipLaunchKernelGGL((job_kernel<2, SRC, DST, GATE>), g, blk, 0, st, gd, P, io); break;
    case 4: hipLaunchKernelGGL((job_kernel<4, SRC, DST, GATE>), g, blk, 0, st, gd, P, io); break;
    case 8: hipLaunchKernelGGL((job_kernel<8, SRC, DST, GATE>), g, blk, 0, st, gd, P, io); break;
    case 16: hipLaunchKernelGGL((job_kernel<16, SRC, DST, GATE>), g, blk, 0, st, gd, P, io); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_gate(const GateDesc &gd, const DevPtrs &P, int grid, hipStream_t st)
{
    IOPtrs io = {};
    return launch_job<SRC_ARENA, DST_ARENA, true>(gd, P, io, grid, st);
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

/*
 * qcz_oracle.c -- plain CPU oracle for the compressed state-vector simulator
 * of Wu et al., "Full-State Quantum Circuit Simulation by Using Data
 * Compression" (SC'19).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library under
 * paper_1911_04034_amd/) includes, links or calls this file; only the tests,
 * the smoke check and the CPU-baseline leg of the benchmark load it.  It shares
 * no code with the GPU path: every routine here is written out a second time,
 * slowly and directly, so that the two can be compared byte for byte.
 *
 * What it computes, in the paper's terms:
 *   - gates on a 2^n complex128 state (Sec. 2.1, Eq. (5); Sec. 3.1, Eqs. (6)
 *     and (7)); qubit k is bit k of the amplitude index;
 *   - Solution C of Sec. 4.2: bit-plane truncation to Sig_Bit_Count bits
 *     (Eq. (12)) and the XOR leading-byte reduction with a two-bit code per
 *     value, followed by a lossless stage (the paper's Zstd role, here the
 *     project's own chunk modes CONST2 / PACK / SPARSE);
 *   - the blockwise loop of Sec. 3.1/3.3: decompress at most two units,
 *     update the amplitude pairs, recompress, move on; control bits that fall
 *     on unit-index bits skip whole units (Sec. 3.3);
 *   - the variable error bound of Sec. 3.7 (start lossless, relax through
 *     1e-5 .. 1e-1 whenever the compressed state does not fit the budget) and
 *     the fidelity lower bound prod(1 - delta_i) of Sec. 3.8, Eq. (11).
 *
 * Readings where the paper is silent (all listed in the design notes):
 *   - the unit of compression is a "chunk" of C interleaved doubles
 *     (C = min(2048, 2b)); a "block" of b amplitudes groups chunks and carries
 *     the error level;
 *   - truncation is toward zero by masking (Sec. 3.7 range (|D(1-d)|, |D|]);
 *     the relative bound applies to each real and imaginary double;
 *   - XOR is taken against the previous *truncated* value; the two-bit code is
 *     the number (0..3) of identical leading bytes, most significant first;
 *   - a chunk holding a subnormal double is stored lossless;
 *   - the lossless stage is the project-defined chunk format described at
 *     oq_encode_chunk (Zstd is not reproducible bit-exactly on a GPU).
 *
 * Gate arithmetic uses an explicit, fixed fused-multiply-add order (see lin2
 * and dmul) so that its results are reproducible to the bit; it must be
 * compiled with -ffp-contract=off.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* Error levels, Sec. 3.7: lossless, then 1e-5, 1e-4, 1e-3, 1e-2, 1e-1.       */
/* ------------------------------------------------------------------------- */
#define OQ_NLEVELS 6
static const double oq_delta_tab[OQ_NLEVELS] = {0.0, 1e-5, 1e-4, 1e-3, 1e-2, 1e-1};

double oq_level_delta(int level)
{
    if (level < 0 || level >= OQ_NLEVELS) return -1.0;
    return oq_delta_tab[level];
}

/* EXP(eps) of Eq. (12): the IEEE-754 exponent of eps, eps = 1.f * 2^EXP. */
int oq_exp_of(double eps)
{
    int e;
    frexp(eps, &e);          /* eps = m * 2^e with m in [0.5, 1) */
    return e - 1;
}

/* Sig_Bit_Count of Eq. (12) for binary64: 12 sign+exponent bits - EXP(eps).
 * Level 0 (lossless) keeps all 64 bits. */
int oq_sig_bits(int level)
{
    if (level <= 0) return 64;
    return 12 - oq_exp_of(oq_delta_tab[level]);
}

static uint64_t dbits(double x) { uint64_t b; memcpy(&b, &x, 8); return b; }
static double bitsd(uint64_t b) { double x; memcpy(&x, &b, 8); return x; }

/* Bit-plane truncation: keep the K most significant bits, zero the rest. */
uint64_t oq_truncate_bits(uint64_t b, int K)
{
    if (K >= 64) return b;
    return b & ~((UINT64_C(1) << (64 - K)) - 1);
}

double oq_truncate(double x, int level)
{
    return bitsd(oq_truncate_bits(dbits(x), oq_sig_bits(level)));
}

static int is_subnormal(uint64_t b)
{
    return ((b >> 52) & 0x7FF) == 0 && (b & ((UINT64_C(1) << 52) - 1)) != 0;
}

/* ------------------------------------------------------------------------- */
/* Bit streams: bit p of a stream lives in byte p/8 at bit p%8 (LSB first);  */
/* a field of r bits is stored least significant bit first.                   */
/* ------------------------------------------------------------------------- */
static void put_bits(uint8_t *buf, uint64_t *pos, uint64_t v, int nbits)
{
    for (int k = 0; k < nbits; ++k) {
        uint64_t p = *pos + (uint64_t)k;
        if ((v >> k) & 1u) buf[p >> 3] |= (uint8_t)(1u << (p & 7));
    }
    *pos += (uint64_t)nbits;
}

static uint64_t get_bits(const uint8_t *buf, uint64_t pos, int nbits)
{
    uint64_t v = 0;
    for (int k = 0; k < nbits; ++k) {
        uint64_t p = pos + (uint64_t)k;
        if ((buf[p >> 3] >> (p & 7)) & 1u) v |= UINT64_C(1) << k;
    }
    return v;
}

static void put_u32(uint8_t *p, uint32_t v) { for (int k = 0; k < 4; ++k) p[k] = (uint8_t)(v >> (8 * k)); }
static void put_u64(uint8_t *p, uint64_t v) { for (int k = 0; k < 8; ++k) p[k] = (uint8_t)(v >> (8 * k)); }
static uint32_t get_u32(const uint8_t *p) { uint32_t v = 0; for (int k = 0; k < 4; ++k) v |= (uint32_t)p[k] << (8 * k); return v; }
static uint64_t get_u64(const uint8_t *p) { uint64_t v = 0; for (int k = 0; k < 8; ++k) v |= (uint64_t)p[k] << (8 * k); return v; }

/* ------------------------------------------------------------------------- */
/* Solution C, step "XOR leading-zero data reduction" (Sec. 4.2).            */
/* ------------------------------------------------------------------------- */

/* Number of identical leading bytes (most significant first) of two values,
 * capped at 3 so that it fits the two-bit code. */
static int lead_bytes(uint64_t cur, uint64_t prev)
{
    uint64_t d = cur ^ prev;
    int L = 0;
    while (L < 3 && ((d >> (56 - 8 * L)) & 0xFFu) == 0) ++L;
    return L;
}

/* Residual bits of a value whose first L bytes repeat the previous value:
 * the significant bits that remain after those bytes. */
static int resid_bits(int K, int L)
{
    int r = K - 8 * L;
    return r > 0 ? r : 0;
}

static uint64_t top_mask(int nbits)
{
    if (nbits <= 0) return 0;
    if (nbits >= 64) return ~UINT64_C(0);
    return ~UINT64_C(0) << (64 - nbits);
}

/* ------------------------------------------------------------------------- */
/* Chunk format.                                                              */
/*                                                                            */
/* A chunk holds C doubles v_0..v_{C-1} = re a_0, im a_0, re a_1, ... of C/2   */
/* consecutive amplitudes.  Bytes, little-endian:                             */
/*   u32 header: bits 0-1 mode, bits 2-4 level index (0 lossless, 1..5),     */
/*               bits 5-31 zero.                                              */
/*   mode CONST2 (1): t_0 (u64), t_1 (u64).  Used when every even value      */
/*               equals t_0 and every odd value equals t_1.                   */
/*   mode PACK (0): codes area of 4*ceil(C/16) bytes (value i's two-bit code  */
/*               L_i at bit 2i), then the residual stream: for each value in */
/*               order, r_i = max(0, K - 8 L_i) bits holding the low r_i bits */
/*               of its K-bit significant prefix; zero-padded to a byte.      */
/*   mode SPARSE (2): bitmap of 4*ceil(C/32) bytes (bit i set when t_i has   */
/*               any bit set), then a PACK body (codes area of               */
/*               4*ceil(nnz/16) bytes and residual stream) over the          */
/*               subsequence of nonzero values, XOR-chained among themselves. */
/* The chain starts from t_{-1} = 0.  The encoder picks CONST2 when it        */
/* applies, otherwise the smaller of PACK and SPARSE (PACK on a tie).         */
/* ------------------------------------------------------------------------- */
#define OQ_MODE_PACK 0
#define OQ_MODE_CONST2 1
#define OQ_MODE_SPARSE 2

size_t oq_chunk_cap(int C)
{
    return 4 + 4 * (size_t)((C + 15) / 16) + 8 * (size_t)C;
}

/* Size in bytes of a PACK body (codes + residual) over the sequence s[0..N). */
static size_t pack_body_size(const uint64_t *s, int N, int K)
{
    uint64_t bits = 0, prev = 0;
    for (int i = 0; i < N; ++i) {
        bits += (uint64_t)resid_bits(K, lead_bytes(s[i], prev));
        prev = s[i];
    }
    return 4 * (size_t)((N + 15) / 16) + (size_t)((bits + 7) / 8);
}

/* Write a PACK body over s[0..N) at out; returns its size. */
static size_t pack_body_write(const uint64_t *s, int N, int K, uint8_t *out)
{
    size_t codes_bytes = 4 * (size_t)((N + 15) / 16);
    uint8_t *res = out + codes_bytes;
    uint64_t cpos = 0, rpos = 0, prev = 0;
    for (int i = 0; i < N; ++i) {
        int L = lead_bytes(s[i], prev);
        int r = resid_bits(K, L);
        put_bits(out, &cpos, (uint64_t)L, 2);
        if (r > 0) {
            uint64_t sig = (K >= 64) ? s[i] : (s[i] >> (64 - K));
            uint64_t R = (r >= 64) ? sig : (sig & ((UINT64_C(1) << r) - 1));
            put_bits(res, &rpos, R, r);
        }
        prev = s[i];
    }
    return codes_bytes + (size_t)((rpos + 7) / 8);
}

/* Read a PACK body of N values; returns bytes consumed or 0 on error. */
static size_t pack_body_read(const uint8_t *in, size_t avail, int N, int K, uint64_t *s)
{
    size_t codes_bytes = 4 * (size_t)((N + 15) / 16);
    if (codes_bytes > avail) return 0;
    const uint8_t *res = in + codes_bytes;
    size_t res_avail = avail - codes_bytes;
    uint64_t rpos = 0, prev = 0;
    for (int i = 0; i < N; ++i) {
        int L = (int)get_bits(in, 2 * (uint64_t)i, 2);
        int r = resid_bits(K, L);
        if ((rpos + (uint64_t)r + 7) / 8 > res_avail) return 0;
        uint64_t R = get_bits(res, rpos, r);
        rpos += (uint64_t)r;
        uint64_t low = (K >= 64) ? R : (R << (64 - K));
        s[i] = (prev & top_mask(8 * L)) | low;
        prev = s[i];
    }
    return codes_bytes + (size_t)((rpos + 7) / 8);
}

/* ------------------------------------------------------------------------- */
/* Entropy stage (the entropy-coding role of Zstd in Solution C, Sec. 4.2).  */
/*                                                                            */
/* A PACK or SPARSE body may carry its residuals entropy-coded; header bit 5  */
/* (E) says so.  The residual of value i (its significant prefix after the    */
/* L_i leading bytes it shares with the previous value) is cut into 4-bit     */
/* lanes: lane j holds bits [64-4j-w_j, 64-4j) of the value, w_j =            */
/* min(4, K-4j), j = 0 .. NN-1 with NN = ceil(K/4); value i codes the lanes   */
/* j >= 2 L_i (the lanes of its shared bytes are copied from the previous     */
/* value).  Each lane has its own code:                                       */
/*   RAW   (0): the w_j-bit symbol as a field;                                */
/*   CONST (1): every symbol of the lane is one value, stored once in the     */
/*              table; nothing per value;                                     */
/*   CODED (2): a canonical Huffman code (Huffman 1952) over the lane's        */
/*              2^w_j symbols, code lengths limited to 8 bits.                */
/* E body, after the codes area of the PACK / SPARSE body:                   */
/*   u32 lane word: mode of lane j at bits 2j..2j+1 (0 for j >= NN);          */
/*   table: a 4-bit-nibble sequence (nibble k at bits 4(k%2) of byte k/2):    */
/*          for each lane in order, CONST: its symbol; CODED: the code length */
/*          (0 = symbol absent) of each of its 2^w_j symbols; zero-padded to  */
/*          a multiple of 4 bytes;                                            */
/*   sub-stream lengths: ceil(C/16) fields of 12 bits, LSB first: field s is  */
/*          the bit length of sub-stream s; zero-padded to 4 bytes;          */
/*   bit stream, LSB first: sub-streams 0, 1, ... back to back; sub-stream s  */
/*          holds the coded lanes of the stored values at chunk positions     */
/*          16s .. 16s+15, value by value in position order, lanes in         */
/*          increasing j.  A RAW symbol is a w_j-bit field; a CODED symbol is */
/*          its canonical code written first bit first (bit-reversed into the */
/*          LSB-first stream); zero-padded to a byte.                         */
/* Lane choice (encoder), from the lane's n_j symbols and their counts:       */
/*   RAW when n_j = 0; CONST when one distinct symbol and 4 < n_j w_j; CODED  */
/*   when at least two distinct symbols, the most frequent one has at least   */
/*   twice the uniform share (max count * 2^w_j >= 2 n_j) and                 */
/*   4 * 2^w_j + sum(count * length) < n_j w_j; otherwise RAW.               */
/* Chunk choice: CONST2 when it applies; else the smaller of PACK and SPARSE  */
/* (PACK on a tie) as before; with the entropy stage enabled, that body is    */
/* entropy-coded when the result is strictly smaller.                         */
/* ------------------------------------------------------------------------- */
#define OQ_HDR_ENT 0x20u
#define OQ_ENC_ENTROPY 1    /* consider the entropy-coded body */
#define OQ_ENC_FORCE_ENT 2  /* test hook: always entropy-code the PACK / SPARSE body */
#define OQ_ENC_FORCE_CODED 4 /* test hook (with OQ_ENC_FORCE_ENT): every lane with two or more distinct
                                symbols CODED, with one CONST, without the cost comparisons */
#define OQ_HUFF_MAXLEN 8
enum { OQ_LANE_RAW = 0, OQ_LANE_CONST = 1, OQ_LANE_CODED = 2 };

/* ------------------------------------------------------------------------- */
/* Solution D of Sec. 4.2: the real and imaginary parts are separated before  */
/* the Solution C steps.  Header bit 6 (R) marks a PACK or SPARSE stream      */
/* whose values are stored in the order re a_0, re a_1, ..., re a_{A-1},      */
/* im a_0, ..., im a_{A-1} (A = C/2 amplitudes) instead of interleaved; every */
/* step after the reordering (XOR chain, truncation, codes, bitmap, entropy   */
/* stage) runs on that sequence unchanged.  CONST2 is defined on amplitudes   */
/* and never carries R.                                                       */
/* ------------------------------------------------------------------------- */
#define OQ_HDR_RSH 0x40u
#define OQ_ENC_RESHUFFLE 8  /* store PACK / SPARSE values re parts first, then im parts (Solution D) */

/* stored position j -> interleaved position */
static int rsh_pos(int j, int C) { return j < C / 2 ? 2 * j : 2 * (j - C / 2) + 1; }

static int nib_lanes(int K) { return (K + 3) / 4; }
static int lane_width(int K, int j) { int w = K - 4 * j; return w < 4 ? w : 4; }
static unsigned lane_symbol(uint64_t t, int K, int j)
{
    int w = lane_width(K, j);
    return (unsigned)((t >> (64 - 4 * j - w)) & ((1u << w) - 1u));
}

/* Huffman code lengths (Huffman 1952) for the symbols with cnt > 0 (at least
 * two of them).  Leaves in increasing (count, symbol) order; internal nodes in
 * creation order form a second queue whose weights never decrease, so each
 * step joins the two smallest heads, taking the leaf when a leaf and a node
 * weigh the same.  A code length is the depth of the leaf.  Lengths above
 * OQ_HUFF_MAXLEN are cut to it, then, while the Kraft sum exceeds 1, the
 * longest code below the limit (fewest occurrences, then lowest symbol, on
 * ties) is made one bit longer. */
static void huff_lengths(const uint32_t *cnt, int nsym, uint8_t *len)
{
    int leaf[16], nl = 0;
    for (int sy = 0; sy < nsym; ++sy) {
        len[sy] = 0;
        if (cnt[sy] > 0) leaf[nl++] = sy;
    }
    for (int a = 1; a < nl; ++a) {          /* insertion sort by (count, symbol) */
        int v = leaf[a], b = a - 1;
        while (b >= 0 && (cnt[leaf[b]] > cnt[v] || (cnt[leaf[b]] == cnt[v] && leaf[b] > v))) {
            leaf[b + 1] = leaf[b];
            --b;
        }
        leaf[b + 1] = v;
    }
    uint64_t w[32];
    int parent[32], depth[32];
    for (int i = 0; i < nl; ++i) w[i] = cnt[leaf[i]];
    int nextleaf = 0, nextnode = nl, nn = nl;
    while (nn < 2 * nl - 1) {
        int pick[2];
        for (int k = 0; k < 2; ++k) {
            int take_leaf;
            if (nextleaf < nl && nextnode < nn) take_leaf = w[nextleaf] <= w[nextnode];
            else take_leaf = nextleaf < nl;
            pick[k] = take_leaf ? nextleaf++ : nextnode++;
        }
        w[nn] = w[pick[0]] + w[pick[1]];
        parent[pick[0]] = nn;
        parent[pick[1]] = nn;
        ++nn;
    }
    depth[nn - 1] = 0;
    for (int i = nn - 2; i >= 0; --i) depth[i] = depth[parent[i]] + 1;
    int maxl = 0;
    for (int i = 0; i < nl; ++i) {
        len[leaf[i]] = (uint8_t)depth[i];
        if (depth[i] > maxl) maxl = depth[i];
    }
    if (maxl <= OQ_HUFF_MAXLEN) return;
    for (int sy = 0; sy < nsym; ++sy)
        if (len[sy] > OQ_HUFF_MAXLEN) len[sy] = OQ_HUFF_MAXLEN;
    for (;;) {
        uint32_t kraft = 0;   /* in units of 2^-8 */
        for (int sy = 0; sy < nsym; ++sy)
            if (len[sy]) kraft += 1u << (OQ_HUFF_MAXLEN - len[sy]);
        if (kraft <= (1u << OQ_HUFF_MAXLEN)) break;
        int best = -1;
        for (int sy = 0; sy < nsym; ++sy) {
            if (!len[sy] || len[sy] >= OQ_HUFF_MAXLEN) continue;
            if (best < 0 || len[sy] > len[best] || (len[sy] == len[best] && cnt[sy] < cnt[best])) best = sy;
        }
        len[best] += 1;
    }
}

/* Canonical codes for lengths len[] (0 = absent): symbols in increasing
 * (length, symbol) order take consecutive codes, each shifted left by the
 * growth of the length (the first takes 0). */
static void canon_codes(const uint8_t *len, int nsym, uint32_t *code)
{
    uint32_t c = 0;
    int prev = 0, first = 1;
    for (int l = 1; l <= OQ_HUFF_MAXLEN; ++l)
        for (int sy = 0; sy < nsym; ++sy) {
            if (len[sy] != l) continue;
            if (first) { c = 0; first = 0; }
            else c = (c + 1) << (l - prev);
            code[sy] = c;
            prev = l;
        }
}

static uint32_t bit_reverse(uint32_t v, int n)
{
    uint32_t r = 0;
    for (int k = 0; k < n; ++k) r |= ((v >> k) & 1u) << (n - 1 - k);
    return r;
}

typedef struct {
    int mode;
    unsigned csym;            /* CONST: the symbol */
    uint8_t len[16];          /* CODED: code length per symbol */
    uint32_t code[16];        /* CODED: canonical code per symbol */
} oq_lane;

/* Two-bit codes of the XOR chain over s[0..N) (the chain starts from 0). */
static void chain_codes(const uint64_t *s, int N, int *L)
{
    uint64_t prev = 0;
    for (int i = 0; i < N; ++i) {
        L[i] = lead_bytes(s[i], prev);
        prev = s[i];
    }
}

/* Size of the entropy-coded body over s[0..N) (positions pos[] in a chunk of
 * C values), and, when out is not NULL, its bytes. */
static size_t sub_count(int C) { return (size_t)(C + 15) / 16; }
static size_t sub_area(int C) { return 4 * ((12 * sub_count(C) + 31) / 32); }

static size_t ent_body(const uint64_t *s, const int *pos, int N, int C, int K, int flags, uint8_t *out)
{
    int NN = nib_lanes(K);
    int *L = (int *)malloc(sizeof(int) * (size_t)(N > 0 ? N : 1));
    chain_codes(s, N, L);
    uint32_t cnt[16][16];
    uint32_t nj[16];
    memset(cnt, 0, sizeof cnt);
    memset(nj, 0, sizeof nj);
    for (int i = 0; i < N; ++i)
        for (int j = 2 * L[i]; j < NN; ++j) {
            cnt[j][lane_symbol(s[i], K, j)] += 1;
            nj[j] += 1;
        }
    oq_lane lane[16];
    uint64_t bits = 0, nib = 0;
    for (int j = 0; j < NN; ++j) {
        int w = lane_width(K, j), nsym = 1 << w;
        oq_lane *ln = &lane[j];
        memset(ln, 0, sizeof *ln);
        uint64_t raw = (uint64_t)nj[j] * (uint64_t)w;
        int distinct = 0;
        uint32_t mx = 0;
        for (int sy = 0; sy < nsym; ++sy) {
            if (cnt[j][sy]) { ++distinct; ln->csym = (unsigned)sy; }
            if (cnt[j][sy] > mx) mx = cnt[j][sy];
        }
        ln->mode = OQ_LANE_RAW;
        uint64_t cost = raw, tab = 0;
        int forced = (flags & OQ_ENC_FORCE_CODED) != 0;
        if (nj[j] > 0 && distinct == 1) {
            if (4 < raw || forced) { ln->mode = OQ_LANE_CONST; cost = 0; tab = 1; }
        } else if (distinct >= 2 && (forced || (uint64_t)mx * (uint64_t)nsym >= 2ull * nj[j])) {
            huff_lengths(cnt[j], nsym, ln->len);
            uint64_t coded = 4ull * (uint64_t)nsym;
            for (int sy = 0; sy < nsym; ++sy) coded += (uint64_t)cnt[j][sy] * ln->len[sy];
            if (coded < raw || forced) {
                ln->mode = OQ_LANE_CODED;
                canon_codes(ln->len, nsym, ln->code);
                cost = coded - 4ull * (uint64_t)nsym;
                tab = (uint64_t)nsym;
            }
        }
        bits += cost;
        nib += tab;
    }
    size_t codes_bytes = 4 * (size_t)((N + 15) / 16);
    size_t tab_bytes = 4 * (size_t)((nib + 7) / 8);
    size_t sub_bytes = sub_area(C);
    size_t size = codes_bytes + 4 + tab_bytes + sub_bytes + (size_t)((bits + 7) / 8);
    if (out) {
        uint64_t p = 0;
        for (int i = 0; i < N; ++i) put_bits(out, &p, (uint64_t)L[i], 2);
        uint8_t *lw = out + codes_bytes;
        uint32_t word = 0;
        for (int j = 0; j < NN; ++j) word |= (uint32_t)lane[j].mode << (2 * j);
        put_u32(lw, word);
        uint8_t *tb = lw + 4;
        uint64_t tp = 0;
        for (int j = 0; j < NN; ++j) {
            int nsym = 1 << lane_width(K, j);
            if (lane[j].mode == OQ_LANE_CONST) put_bits(tb, &tp, lane[j].csym, 4);
            else if (lane[j].mode == OQ_LANE_CODED)
                for (int sy = 0; sy < nsym; ++sy) put_bits(tb, &tp, lane[j].len[sy], 4);
        }
        uint8_t *sl = tb + tab_bytes;
        uint8_t *bs = sl + sub_bytes;
        uint64_t bp = 0, lp = 0;
        int i = 0;
        for (int sub = 0; sub < (int)sub_count(C); ++sub) {
            uint64_t start = bp;
            while (i < N && pos[i] < 16 * (sub + 1)) {
                for (int j = 2 * L[i]; j < NN; ++j) {
                    unsigned sy = lane_symbol(s[i], K, j);
                    if (lane[j].mode == OQ_LANE_RAW) put_bits(bs, &bp, sy, lane_width(K, j));
                    else if (lane[j].mode == OQ_LANE_CODED)
                        put_bits(bs, &bp, bit_reverse(lane[j].code[sy], lane[j].len[sy]), lane[j].len[sy]);
                }
                ++i;
            }
            put_bits(sl, &lp, bp - start, 12);
        }
    }
    free(L);
    return size;
}

/* Read an entropy-coded body of N values at positions pos[] of a chunk of C
 * values; returns the bytes it occupies, 0 when malformed. */
static size_t ent_body_read(const uint8_t *in, size_t avail, const int *pos, int N, int C, int K, uint64_t *s)
{
    int NN = nib_lanes(K);
    size_t codes_bytes = 4 * (size_t)((N + 15) / 16);
    if (codes_bytes + 4 > avail) return 0;
    uint32_t word = get_u32(in + codes_bytes);
    oq_lane lane[16];
    size_t nib = 0;
    for (int j = 0; j < 16; ++j) {
        int m = (int)((word >> (2 * j)) & 3u);
        if (j >= NN) { if (m) return 0; continue; }
        if (m > OQ_LANE_CODED) return 0;
        memset(&lane[j], 0, sizeof lane[j]);
        lane[j].mode = m;
        nib += m == OQ_LANE_CONST ? 1 : m == OQ_LANE_CODED ? (size_t)1 << lane_width(K, j) : 0;
    }
    size_t tab_bytes = 4 * ((nib + 7) / 8);
    size_t sub_bytes = sub_area(C);
    size_t head = codes_bytes + 4 + tab_bytes + sub_bytes;
    if (head > avail) return 0;
    const uint8_t *tb = in + codes_bytes + 4;
    uint64_t tp = 0;
    for (int j = 0; j < NN; ++j) {
        int nsym = 1 << lane_width(K, j);
        if (lane[j].mode == OQ_LANE_CONST) {
            lane[j].csym = (unsigned)get_bits(tb, tp, 4);
            tp += 4;
            if (lane[j].csym >= (unsigned)nsym) return 0;
        } else if (lane[j].mode == OQ_LANE_CODED) {
            uint32_t kraft = 0;
            for (int sy = 0; sy < nsym; ++sy) {
                lane[j].len[sy] = (uint8_t)get_bits(tb, tp, 4);
                tp += 4;
                if (lane[j].len[sy] > OQ_HUFF_MAXLEN) return 0;
                if (lane[j].len[sy]) kraft += 1u << (OQ_HUFF_MAXLEN - lane[j].len[sy]);
            }
            if (kraft == 0 || kraft > (1u << OQ_HUFF_MAXLEN)) return 0;
            canon_codes(lane[j].len, nsym, lane[j].code);
        }
    }
    const uint8_t *sl = in + codes_bytes + 4 + tab_bytes;
    const uint8_t *bs = sl + sub_bytes;
    size_t bs_avail = avail - head;
    uint64_t bp = 0, prev = 0;
    int i = 0;
    for (int sub = 0; sub < (int)sub_count(C); ++sub) {
        uint64_t want = get_bits(sl, 12 * (uint64_t)sub, 12), start = bp;
        while (i < N && pos[i] < 16 * (sub + 1)) {
            int Li = (int)get_bits(in, 2 * (uint64_t)i, 2);
            uint64_t v = prev & top_mask(8 * Li);
            for (int j = 2 * Li; j < NN; ++j) {
                int w = lane_width(K, j);
                unsigned sy;
                if (lane[j].mode == OQ_LANE_RAW) {
                    if ((bp + (uint64_t)w + 7) / 8 > bs_avail) return 0;
                    sy = (unsigned)get_bits(bs, bp, w);
                    bp += (uint64_t)w;
                } else if (lane[j].mode == OQ_LANE_CONST) {
                    sy = lane[j].csym;
                } else {
                    /* read the code first bit first until it names a symbol */
                    uint32_t acc = 0;
                    int l = 0, found = -1;
                    while (found < 0) {
                        if (l == OQ_HUFF_MAXLEN || (bp + 8) / 8 > bs_avail) return 0;
                        acc = (acc << 1) | (uint32_t)get_bits(bs, bp, 1);
                        ++bp;
                        ++l;
                        for (int t = 0; t < (1 << w); ++t)
                            if (lane[j].len[t] == l && lane[j].code[t] == acc) { found = t; break; }
                    }
                    sy = (unsigned)found;
                }
                v |= (uint64_t)sy << (64 - 4 * j - w);
            }
            s[i] = v;
            prev = v;
            ++i;
        }
        if (bp - start != want) return 0;
    }
    if (i != N) return 0;
    return head + (size_t)((bp + 7) / 8);
}

/* Exported for the pins of the code construction: lengths (0 for absent
 * symbols) of at least two symbols with counts (nsym <= 16), and canonical
 * codes for given lengths.  Return -1 on bad arguments. */
int oq_huff_lengths(const uint32_t *cnt, int nsym, uint8_t *len)
{
    int present = 0;
    if (nsym < 1 || nsym > 16) return -1;
    for (int sy = 0; sy < nsym; ++sy) present += cnt[sy] > 0;
    if (present < 2) return -1;
    huff_lengths(cnt, nsym, len);
    return 0;
}

int oq_canon_codes(const uint8_t *len, int nsym, uint32_t *code)
{
    if (nsym < 1 || nsym > 16) return -1;
    for (int sy = 0; sy < nsym; ++sy) {
        code[sy] = 0;
        if (len[sy] > OQ_HUFF_MAXLEN) return -1;
    }
    canon_codes(len, nsym, code);
    return 0;
}

/* Encode one chunk of C doubles at error level `level` with codec flags
 * (OQ_ENC_*); returns its size.  `out` must hold oq_chunk_cap(C) bytes, or
 * oq_chunk_cap_forced(C) with OQ_ENC_FORCE_ENT. */
size_t oq_encode_chunk_ex(const double *x, int C, int level, int flags, uint8_t *out);

size_t oq_chunk_cap_forced(int C)
{
    return 4 + 4 * (size_t)((C + 31) / 32) + 4 * (size_t)((C + 15) / 16) + 4 + 128 + sub_area(C) + 16 * (size_t)C;
}

/* Encode one chunk of C doubles at error level `level`; returns its size.
 * `out` must hold oq_chunk_cap(C) bytes. */
size_t oq_encode_chunk(const double *x, int C, int level, uint8_t *out)
{
    return oq_encode_chunk_ex(x, C, level, 0, out);
}

size_t oq_encode_chunk_ex(const double *x, int C, int level, int flags, uint8_t *out)
{
    if (C < 4 || (C & (C - 1)) != 0 || level < 0 || level >= OQ_NLEVELS) return 0;
    int lev = level;
    for (int i = 0; i < C; ++i)
        if (is_subnormal(dbits(x[i]))) lev = 0;
    int K = oq_sig_bits(lev);

    uint64_t *t = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)C);
    uint64_t *nz = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)C);
    for (int i = 0; i < C; ++i) t[i] = oq_truncate_bits(dbits(x[i]), K);

    int force = (flags & OQ_ENC_FORCE_ENT) != 0;
    int hooks = flags & OQ_ENC_FORCE_CODED;
    memset(out, 0, force ? oq_chunk_cap_forced(C) : oq_chunk_cap(C));
    size_t size;
    int const2 = 1;
    for (int i = 0; i < C; ++i)
        if (t[i] != t[i & 1]) const2 = 0;
    if (const2 && !force) {
        put_u32(out, (uint32_t)(OQ_MODE_CONST2 | (lev << 2)));
        put_u64(out + 4, t[0]);
        put_u64(out + 12, t[1]);
        size = 20;
    } else {
        int rsh = (flags & OQ_ENC_RESHUFFLE) != 0;
        if (rsh) {   /* Solution D: the values in stored order */
            uint64_t *u = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)C);
            for (int j = 0; j < C; ++j) u[j] = t[rsh_pos(j, C)];
            memcpy(t, u, sizeof(uint64_t) * (size_t)C);
            free(u);
        }
        int nnz = 0;
        int *pos = (int *)malloc(sizeof(int) * (size_t)C);
        int *allpos = (int *)malloc(sizeof(int) * (size_t)C);
        for (int i = 0; i < C; ++i) {
            allpos[i] = i;
            if (t[i] != 0) { pos[nnz] = i; nz[nnz++] = t[i]; }
        }
        size_t bitmap_bytes = 4 * (size_t)((C + 31) / 32);
        size_t pack_size = 4 + pack_body_size(t, C, K);
        size_t sparse_size = 4 + bitmap_bytes + pack_body_size(nz, nnz, K);
        int sparse = sparse_size < pack_size;
        size_t base = sparse ? sparse_size : pack_size;
        size_t lead = sparse ? 4 + bitmap_bytes : 4;
        int ent = 0;
        if (flags & (OQ_ENC_ENTROPY | OQ_ENC_FORCE_ENT)) {
            size_t esize = lead + (sparse ? ent_body(nz, pos, nnz, C, K, hooks, NULL)
                                          : ent_body(t, allpos, C, C, K, hooks, NULL));
            ent = force || esize < base;
        }
        uint32_t hdr = (uint32_t)((sparse ? OQ_MODE_SPARSE : OQ_MODE_PACK) | (lev << 2)) | (ent ? OQ_HDR_ENT : 0u) |
                       (rsh ? OQ_HDR_RSH : 0u);
        put_u32(out, hdr);
        if (sparse) {
            uint64_t bpos = 0;
            for (int i = 0; i < C; ++i) put_bits(out + 4, &bpos, t[i] != 0, 1);
        }
        if (ent) size = lead + (sparse ? ent_body(nz, pos, nnz, C, K, hooks, out + lead)
                                       : ent_body(t, allpos, C, C, K, hooks, out + lead));
        else size = lead + (sparse ? pack_body_write(nz, nnz, K, out + lead) : pack_body_write(t, C, K, out + lead));
        free(pos);
        free(allpos);
    }
    free(t);
    free(nz);
    return size;
}

/* ------------------------------------------------------------------------- */
/* Solution B of Sec. 4.2 (prediction-based, complex-aware): every value is   */
/* quantized in the logarithmic domain, predicted from the previous value of  */
/* the same part (real parts from real parts, imaginary from imaginary), and  */
/* the quantization codes (16,384 bins) are Huffman coded.                     */
/*                                                                            */
/* Log transform: the IEEE-754 bit pattern of |x|, read as an integer v (the  */
/* bits without the sign), grows like 2^52 log2|x| (a piecewise-linear        */
/* logarithm); one step of v changes |x| by at most a factor 1 + 2^-52.  The  */
/* sign travels as one bit beside the code.  Quantization at level l:         */
/* k = floor((v + W/2) / W) with bin                                          */
/* width W = 2^w, w = 52 - t_l, t = 16, 13, 9, 6, 3 for 1e-5 .. 1e-1 (the     */
/* largest t with 2^-(t+1) <= epsilon); the value is rebuilt from k W, which  */
/* is within W/2 steps of v: relative error at most 2^-(t+1) <= epsilon.      */
/* Prediction (Lorenzo in one dimension, on the quantized integers): the code */
/* of value j is k_j - k_p, p the previous value of its part that was not     */
/* zero (k_p = 0 before the first).  Quantizing before predicting makes every */
/* code depend on the input values only (the dual quantization of GPU         */
/* prediction compressors), with the same bound as predicting from rebuilt    */
/* values.  Symbols: 0 escape (the value stored verbatim: a first value, a    */
/* code outside the bins, a subnormal, inf or NaN, or k W beyond the finite   */
/* range), 1 an exact zero, 2 + (code + 8190) for codes in [-8190, 8191];    */
/* every symbol but the escape is followed by the value's sign bit.           */
/* Lossy levels only (level 0 has no bins).                                   */
/*                                                                            */
/* Stream (mode 3 in the header, bits 5 and 6 zero), coding order re a_0 ..  */
/* re a_{A-1}, im a_0 .. im a_{A-1}, in sub-streams of 32 symbols:            */
/*   u32 header; u16 count of symbols per code length 1..16;                  */
/*   u16 bit length of each of the C/32 sub-streams;                          */
/*   u16 symbols in canonical order (length, then symbol), zero-padded to a   */
/*   4-byte boundary; the codes (canonical, first bit first into an LSB-first */
/*   bit stream, each but an escape's followed by the sign bit, sub-streams   */
/*   back to back), zero-padded to 4 bytes; u64 escaped values in coding      */
/*   order.                                                                   */
/* Code lengths: Huffman over the symbols present (leaves in (count, symbol)  */
/* order, two queues, the leaf first on equal weights); a lone symbol takes   */
/* length 1.  With C <= 2048 values no length exceeds 16 (a depth-17 leaf     */
/* needs a total weight of at least the Fibonacci number F(19) = 4181).       */
/* ------------------------------------------------------------------------- */
#define OQ_MODE_PRED 3
#define OQ_PRED_NSYM 16384
#define OQ_PRED_MAXLEN 16
#define OQ_PRED_SUB 32

static const int oq_pred_t[OQ_NLEVELS] = {0, 16, 13, 9, 6, 3};

int oq_pred_width(int level) { return (level >= 1 && level < OQ_NLEVELS) ? 52 - oq_pred_t[level] : -1; }

static uint64_t pred_v(uint64_t b) { return b & 0x7FFFFFFFFFFFFFFFull; }

/* floor((v + W/2) / W), v < 2^63 (no overflow in 64 unsigned bits) */
static int64_t pred_k(uint64_t v, int w) { return (int64_t)((v + ((uint64_t)1 << (w - 1))) >> w); }

/* a value quantizes when it is a nonzero normal double whose rebuilt value
 * k W is finite */
static int pred_quantizable(uint64_t b, int w)
{
    uint64_t e = (b >> 52) & 0x7FF;
    if (e == 0 || e == 0x7FF) return 0;
    uint64_t m = (uint64_t)pred_k(pred_v(b), w) << w;
    return ((m >> 52) & 0x7FF) != 0x7FF && (m >> 63) == 0;
}

/* Symbols of one chunk in coding order; returns the number of escapes. */
int oq_pred_symbols(const double *x, int C, int level, uint16_t *sym)
{
    int w = oq_pred_width(level), A = C / 2, nesc = 0;
    if (w < 0) return -1;
    for (int part = 0; part < 2; ++part) {
        int64_t kp = 0;
        int have = 0;   /* a previous value of the part that was not zero */
        for (int a = 0; a < A; ++a) {
            uint64_t b = dbits(x[2 * a + part]);
            int j = part * A + a;
            if ((b << 1) == 0) { sym[j] = 1; continue; }          /* +-0: the prediction goes on from k_p */
            int64_t k = pred_k(pred_v(b), w);
            int64_t d = k - kp;
            if (have && pred_quantizable(b, w) && d >= -8190 && d <= 8191) sym[j] = (uint16_t)(2 + (d + 8190));
            else { sym[j] = 0; ++nesc; }
            kp = k;   /* (an escaped value's k is taken from the value itself) */
            have = 1;
        }
    }
    return nesc;
}

typedef struct { uint32_t cnt; int sym; } oq_leaf;

static int leaf_cmp(const void *pa, const void *pb)
{
    const oq_leaf *a = (const oq_leaf *)pa, *b = (const oq_leaf *)pb;
    if (a->cnt != b->cnt) return a->cnt < b->cnt ? -1 : 1;
    return a->sym < b->sym ? -1 : (a->sym > b->sym);
}

/* Huffman code lengths of the symbols with cnt > 0 (cnt over nsym symbols);
 * returns the longest length, or -1 with no symbol present. */
int oq_pred_huff_lengths(const uint32_t *cnt, int nsym, uint8_t *len)
{
    int nl = 0;
    for (int sy = 0; sy < nsym; ++sy) { len[sy] = 0; nl += cnt[sy] > 0; }
    if (nl == 0) return -1;
    oq_leaf *lv = (oq_leaf *)malloc(sizeof(oq_leaf) * (size_t)nl);
    nl = 0;
    for (int sy = 0; sy < nsym; ++sy)
        if (cnt[sy]) { lv[nl].cnt = cnt[sy]; lv[nl].sym = sy; ++nl; }
    qsort(lv, (size_t)nl, sizeof(oq_leaf), leaf_cmp);
    if (nl == 1) { len[lv[0].sym] = 1; free(lv); return 1; }
    uint64_t *wt = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(2 * nl));
    int *parent = (int *)malloc(sizeof(int) * (size_t)(2 * nl));
    int *depth = (int *)malloc(sizeof(int) * (size_t)(2 * nl));
    for (int i = 0; i < nl; ++i) wt[i] = lv[i].cnt;
    int nextleaf = 0, nextnode = nl, nn = nl;
    while (nn < 2 * nl - 1) {
        int pick[2];
        for (int q = 0; q < 2; ++q) {
            int take_leaf;
            if (nextleaf < nl && nextnode < nn) take_leaf = wt[nextleaf] <= wt[nextnode];
            else take_leaf = nextleaf < nl;
            pick[q] = take_leaf ? nextleaf++ : nextnode++;
        }
        wt[nn] = wt[pick[0]] + wt[pick[1]];
        parent[pick[0]] = parent[pick[1]] = nn;
        ++nn;
    }
    depth[nn - 1] = 0;
    for (int i = nn - 2; i >= 0; --i) depth[i] = depth[parent[i]] + 1;
    int maxl = 0;
    for (int i = 0; i < nl; ++i) {
        len[lv[i].sym] = (uint8_t)depth[i];
        if (depth[i] > maxl) maxl = depth[i];
    }
    free(lv); free(wt); free(parent); free(depth);
    return maxl;
}

/* Canonical codes of lengths len[] (0: absent), lengths up to 16. */
static void pred_canon(const uint8_t *len, int nsym, uint32_t *code)
{
    uint32_t c = 0;
    int prev = 0, first = 1;
    for (int l = 1; l <= OQ_PRED_MAXLEN; ++l)
        for (int sy = 0; sy < nsym; ++sy) {
            if (len[sy] != l) continue;
            if (first) { c = 0; first = 0; }
            else c = (c + 1) << (l - prev);
            code[sy] = c;
            prev = l;
        }
}

static size_t pad4s(size_t x) { return (x + 3) & ~(size_t)3; }

size_t oq_pred_cap(int C)
{
    return 4 + 2 * OQ_PRED_MAXLEN + 2 * (size_t)(C / OQ_PRED_SUB) + pad4s(2 * (size_t)C) +
           4 * (size_t)((C * (OQ_PRED_MAXLEN + 1) + 31) / 32) + 8 * (size_t)C;
}

/* Encode one chunk with Solution B at lossy level 1..5; returns its size
 * (0 for a bad size or level).  `out` holds oq_pred_cap(C) bytes. */
size_t oq_encode_pred(const double *x, int C, int level, uint8_t *out)
{
    if (C < 64 || (C & (C - 1)) != 0 || oq_pred_width(level) < 0) return 0;
    int A = C / 2, NS = C / OQ_PRED_SUB;
    uint16_t *sym = (uint16_t *)malloc(sizeof(uint16_t) * (size_t)C);
    int nesc = oq_pred_symbols(x, C, level, sym);
    uint32_t *cnt = (uint32_t *)calloc(OQ_PRED_NSYM, sizeof(uint32_t));
    uint8_t *len = (uint8_t *)malloc(OQ_PRED_NSYM);
    uint32_t *code = (uint32_t *)calloc(OQ_PRED_NSYM, sizeof(uint32_t));
    for (int j = 0; j < C; ++j) cnt[sym[j]] += 1;
    oq_pred_huff_lengths(cnt, OQ_PRED_NSYM, len);
    pred_canon(len, OQ_PRED_NSYM, code);
    memset(out, 0, oq_pred_cap(C));
    put_u32(out, (uint32_t)(OQ_MODE_PRED | (level << 2)));
    size_t o = 4;
    int nsym = 0;
    for (int l = 1; l <= OQ_PRED_MAXLEN; ++l) {
        int c = 0;
        for (int sy = 0; sy < OQ_PRED_NSYM; ++sy) c += len[sy] == l;
        out[o] = (uint8_t)c; out[o + 1] = (uint8_t)(c >> 8);
        o += 2;
        nsym += c;
    }
    size_t sub_o = o;
    o += 2 * (size_t)NS;
    for (int l = 1; l <= OQ_PRED_MAXLEN; ++l)
        for (int sy = 0; sy < OQ_PRED_NSYM; ++sy)
            if (len[sy] == l) { out[o] = (uint8_t)sy; out[o + 1] = (uint8_t)(sy >> 8); o += 2; }
    o = pad4s(o);
    uint64_t bpos = 0;
    for (int i = 0; i < NS; ++i) {
        uint64_t b0 = bpos;
        for (int j = i * OQ_PRED_SUB; j < (i + 1) * OQ_PRED_SUB; ++j) {
            int l = len[sym[j]];
            put_bits(out + o, &bpos, bit_reverse(code[sym[j]], l), l);   /* first code bit at the lowest position */
            if (sym[j] != 0) {
                int a = j < A ? j : j - A, part = j < A ? 0 : 1;
                put_bits(out + o, &bpos, dbits(x[2 * a + part]) >> 63, 1);
            }
        }
        uint32_t sl = (uint32_t)(bpos - b0);
        out[sub_o + 2 * i] = (uint8_t)sl; out[sub_o + 2 * i + 1] = (uint8_t)(sl >> 8);
    }
    o += 4 * (size_t)((bpos + 31) / 32);
    for (int j = 0; j < C; ++j)
        if (sym[j] == 0) {
            int a = j < A ? j : j - A, part = j < A ? 0 : 1;
            put_u64(out + o, dbits(x[2 * a + part]));
            o += 8;
        }
    (void)nesc;
    (void)nsym;
    free(sym); free(cnt); free(len); free(code);
    return o;
}

/* Decode a Solution B stream; 0 on success, -1 when malformed. */
static int decode_pred(const uint8_t *in, size_t len, int C, double *x)
{
    uint32_t hdr = get_u32(in);
    int level = (int)((hdr >> 2) & 7u), w = oq_pred_width(level);
    if ((hdr & 3u) != OQ_MODE_PRED || (hdr >> 5) != 0 || w < 0 || C < 64) return -1;
    int A = C / 2, NS = C / OQ_PRED_SUB;
    size_t o = 4;
    int cntl[OQ_PRED_MAXLEN + 1], nsym = 0;
    if (len < o + 2 * OQ_PRED_MAXLEN + 2 * (size_t)NS) return -1;
    uint64_t kraft = 0;   /* in units of 2^-16 */
    for (int l = 1; l <= OQ_PRED_MAXLEN; ++l) {
        cntl[l] = in[o] | (in[o + 1] << 8);
        o += 2;
        nsym += cntl[l];
        kraft += (uint64_t)cntl[l] << (OQ_PRED_MAXLEN - l);
    }
    if (nsym < 1 || nsym > C || kraft > (1u << OQ_PRED_MAXLEN)) return -1;
    size_t sub_o = o;
    uint64_t total = 0;
    for (int i = 0; i < NS; ++i) total += (uint64_t)(in[sub_o + 2 * i] | (in[sub_o + 2 * i + 1] << 8));
    o += 2 * (size_t)NS;
    if (len < pad4s(o + 2 * (size_t)nsym)) return -1;
    uint8_t *sgn = (uint8_t *)malloc((size_t)C);
    uint16_t *syms = (uint16_t *)malloc(sizeof(uint16_t) * (size_t)nsym);
    for (int i = 0; i < nsym; ++i) {
        syms[i] = (uint16_t)(in[o + 2 * i] | (in[o + 2 * i + 1] << 8));
        if (syms[i] >= OQ_PRED_NSYM) { free(syms); free(sgn); return -1; }
    }
    o = pad4s(o + 2 * (size_t)nsym);
    size_t bits_o = o;
    o += 4 * (size_t)((total + 31) / 32);
    if (len < o) { free(syms); free(sgn); return -1; }
    /* canonical decoding: first code and first symbol index per length */
    uint32_t firstc[OQ_PRED_MAXLEN + 2];
    int firsti[OQ_PRED_MAXLEN + 2];
    uint32_t c = 0;
    int idx = 0;
    for (int l = 1; l <= OQ_PRED_MAXLEN; ++l) {
        firstc[l] = c;
        firsti[l] = idx;
        c = (c + (uint32_t)cntl[l]) << 1;
        idx += cntl[l];
    }
    uint16_t *sym = (uint16_t *)malloc(sizeof(uint16_t) * (size_t)C);
    uint64_t bpos = 0;
    int rc = 0;
    for (int i = 0; i < NS && !rc; ++i) {
        uint64_t end = bpos + (uint64_t)(in[sub_o + 2 * i] | (in[sub_o + 2 * i + 1] << 8));
        for (int j = i * OQ_PRED_SUB; j < (i + 1) * OQ_PRED_SUB && !rc; ++j) {
            uint32_t v = 0;
            int l = 0, found = 0;
            while (!found && l < OQ_PRED_MAXLEN && bpos < end) {
                v = (v << 1) | (uint32_t)get_bits(in + bits_o, bpos++, 1);
                ++l;
                if (cntl[l] && v >= firstc[l] && v - firstc[l] < (uint32_t)cntl[l]) {
                    sym[j] = syms[firsti[l] + (int)(v - firstc[l])];
                    found = 1;
                }
            }
            if (!found) rc = -1;
            else if (sym[j] != 0) {
                if (bpos >= end) rc = -1;
                else sgn[j] = (uint8_t)get_bits(in + bits_o, bpos++, 1);
            }
        }
        if (!rc && bpos != end) rc = -1;
    }
    int64_t kp[2] = {0, 0};
    for (int j = 0; j < C && !rc; ++j) {
        int part = j < A ? 0 : 1, a = j < A ? j : j - A;
        uint64_t b;
        if (sym[j] == 1) { x[2 * a + part] = bitsd((uint64_t)sgn[j] << 63); continue; }
        if (sym[j] == 0) {
            if (o + 8 > len) { rc = -1; break; }
            b = get_u64(in + o);
            o += 8;
            kp[part] = pred_k(pred_v(b), w);
        } else {
            kp[part] += (int64_t)sym[j] - 2 - 8190;
            int64_t lim = (int64_t)1 << (63 - w);
            if (kp[part] >= lim) { rc = -1; break; }   /* beyond any finite value */
            if (kp[part] <= 0) { rc = -1; break; }
            b = ((uint64_t)kp[part] << w) | ((uint64_t)sgn[j] << 63);
        }
        x[2 * a + part] = bitsd(b);
    }
    if (!rc && o != len) rc = -1;
    free(syms);
    free(sym);
    free(sgn);
    return rc;
}

/* Decode one chunk; returns 0 on success, -1 on a malformed stream. */
int oq_decode_chunk(const uint8_t *in, size_t len, int C, double *x)
{
    if (C < 4 || (C & (C - 1)) != 0 || len < 4) return -1;
    uint32_t hdr = get_u32(in);
    if ((hdr & 3u) == OQ_MODE_PRED) return decode_pred(in, len, C, x);
    int mode = (int)(hdr & 3u), lev = (int)((hdr >> 2) & 7u), ent = (hdr & OQ_HDR_ENT) != 0;
    int rsh = (hdr & OQ_HDR_RSH) != 0;
    if ((hdr >> 7) != 0 || lev >= OQ_NLEVELS) return -1;
    int K = oq_sig_bits(lev);
    if (mode == OQ_MODE_CONST2) {
        if (len != 20 || ent || rsh) return -1;
        uint64_t t0 = get_u64(in + 4), t1 = get_u64(in + 12);
        for (int i = 0; i < C; ++i) x[i] = bitsd((i & 1) ? t1 : t0);
        return 0;
    }
    uint64_t *s = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)C);
    int rc = 0;
    int *pos = (int *)malloc(sizeof(int) * (size_t)C);
    if (mode == OQ_MODE_PACK) {
        for (int i = 0; i < C; ++i) pos[i] = i;
        size_t used = ent ? ent_body_read(in + 4, len - 4, pos, C, C, K, s) : pack_body_read(in + 4, len - 4, C, K, s);
        if (used == 0 || used != len - 4) rc = -1;
        else for (int i = 0; i < C; ++i) x[i] = bitsd(s[i]);
    } else if (mode == OQ_MODE_SPARSE) {
        size_t bitmap_bytes = 4 * (size_t)((C + 31) / 32);
        if (len < 4 + bitmap_bytes) { free(s); free(pos); return -1; }
        int nnz = 0;
        for (int i = 0; i < C; ++i)
            if (get_bits(in + 4, (uint64_t)i, 1)) pos[nnz++] = i;
        size_t used = ent ? ent_body_read(in + 4 + bitmap_bytes, len - 4 - bitmap_bytes, pos, nnz, C, K, s)
                          : pack_body_read(in + 4 + bitmap_bytes, len - 4 - bitmap_bytes, nnz, K, s);
        if (used == 0 || used != len - 4 - bitmap_bytes) rc = -1;
        else {
            int k = 0;
            for (int i = 0; i < C; ++i)
                x[i] = get_bits(in + 4, (uint64_t)i, 1) ? bitsd(s[k++]) : 0.0;
        }
    } else {
        rc = -1;
    }
    if (rc == 0 && rsh) {   /* back to interleaved order */
        double *u = (double *)malloc(sizeof(double) * (size_t)C);
        for (int j = 0; j < C; ++j) u[rsh_pos(j, C)] = x[j];
        memcpy(x, u, sizeof(double) * (size_t)C);
        free(u);
    }
    free(s);
    free(pos);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Gates (Sec. 2.1 Eq. (5); Sec. 3.1 Eqs. (6), (7)).                          */
/* ------------------------------------------------------------------------- */
typedef struct {
    uint32_t kind;          /* OQ_U1 .. OQ_MCZ */
    uint32_t target;        /* q (for DIAG2: first qubit) */
    uint32_t target2;       /* DIAG2: second qubit */
    uint32_t reserved;
    uint64_t control_mask;  /* qubits that must all be 1 */
    double m[8];            /* U1: u00,u01,u10,u11 as (re,im); DIAG1: d0,d1; DIAG2: p0..p3 */
} oq_gate;

enum { OQ_U1 = 0, OQ_DIAG1 = 1, OQ_DIAG2 = 2, OQ_X = 3, OQ_MCZ = 4 };

size_t oq_gate_size(void) { return sizeof(oq_gate); }

/* y = u*a + v*b in a fixed fused-multiply-add order. */
static void lin2(double ur, double ui, double vr, double vi,
                 double ar, double ai, double br, double bi,
                 double *yr, double *yi)
{
    *yr = fma(vr, br, fma(-vi, bi, fma(ur, ar, -(ui * ai))));
    *yi = fma(vr, bi, fma(vi, br, fma(ur, ai, ui * ar)));
}

/* y = d*a. */
static void dmul(double dr, double di, double ar, double ai, double *yr, double *yi)
{
    *yr = fma(dr, ar, -(di * ai));
    *yi = fma(dr, ai, di * ar);
}

/* 0 when the gate record is well formed for an n-qubit state. */
int oq_gate_check(const oq_gate *g, int n)
{
    uint64_t all = (n >= 64) ? ~UINT64_C(0) : ((UINT64_C(1) << n) - 1);
    if (g->control_mask & ~all) return -1;
    for (int k = 0; k < 8; ++k)
        if (!isfinite(g->m[k])) return -1;
    switch (g->kind) {
    case OQ_U1:
    case OQ_DIAG1:
    case OQ_X:
        if ((int)g->target >= n) return -1;
        if (g->control_mask & (UINT64_C(1) << g->target)) return -1;
        return 0;
    case OQ_DIAG2:
        if ((int)g->target >= n || (int)g->target2 >= n || g->target == g->target2) return -1;
        if (g->control_mask & ((UINT64_C(1) << g->target) | (UINT64_C(1) << g->target2))) return -1;
        return 0;
    case OQ_MCZ:
        return g->control_mask ? 0 : -1;
    default:
        return -1;
    }
}

/* Phase a diagonal gate gives the amplitude with global index i. */
static void diag_phase(const oq_gate *g, uint64_t i, double *pr, double *pi)
{
    int idx;
    if (g->kind == OQ_DIAG1) idx = (int)((i >> g->target) & 1u);
    else idx = (int)(((i >> g->target2) & 1u) * 2 + ((i >> g->target) & 1u));
    *pr = g->m[2 * idx];
    *pi = g->m[2 * idx + 1];
}

/* Apply a gate to a set of amplitudes psi[2*l], psi[2*l+1], l < nloc, whose
 * global indices are glob(l).  Pairs (Eq. (6)) are formed by flipping the
 * target bit; `partner(l)` gives the local index of that amplitude. */
typedef struct {
    uint64_t base0, base1;  /* global index of local 0 and of local half */
    uint64_t half;          /* nloc/2 when two units are held, else nloc */
    int pair_units;         /* 1: target flips between the two units */
} oq_layout;

static uint64_t glob_index(const oq_layout *lay, uint64_t l)
{
    if (lay->pair_units) return (l < lay->half) ? lay->base0 + l : lay->base1 + (l - lay->half);
    return lay->base0 + l;
}

static void apply_local(const oq_gate *g, double *psi, uint64_t nloc, const oq_layout *lay)
{
    uint64_t cm = g->control_mask;
    for (uint64_t l = 0; l < nloc; ++l) {
        uint64_t i = glob_index(lay, l);
        if ((i & cm) != cm) continue;
        if (g->kind == OQ_U1 || g->kind == OQ_X) {
            if ((i >> g->target) & 1u) continue;                 /* visit each pair from its 0 side */
            uint64_t lj = lay->pair_units ? l + lay->half : l + (UINT64_C(1) << g->target);
            double ar = psi[2 * l], ai = psi[2 * l + 1], br = psi[2 * lj], bi = psi[2 * lj + 1];
            if (g->kind == OQ_X) {
                psi[2 * l] = br; psi[2 * l + 1] = bi; psi[2 * lj] = ar; psi[2 * lj + 1] = ai;
            } else {
                const double *u = g->m;
                double yr, yi, zr, zi;
                lin2(u[0], u[1], u[2], u[3], ar, ai, br, bi, &yr, &yi);
                lin2(u[4], u[5], u[6], u[7], ar, ai, br, bi, &zr, &zi);
                psi[2 * l] = yr; psi[2 * l + 1] = yi; psi[2 * lj] = zr; psi[2 * lj + 1] = zi;
            }
        } else if (g->kind == OQ_DIAG1 || g->kind == OQ_DIAG2) {
            double pr, pi, yr, yi;
            diag_phase(g, i, &pr, &pi);
            dmul(pr, pi, psi[2 * l], psi[2 * l + 1], &yr, &yi);
            psi[2 * l] = yr; psi[2 * l + 1] = yi;
        } else if (g->kind == OQ_MCZ) {
            psi[2 * l] = -psi[2 * l];
            psi[2 * l + 1] = -psi[2 * l + 1];
        }
    }
}

/* Uncompressed reference: apply one gate to the full state psi (2*2^n doubles). */
int oq_apply_gate_dense(double *psi, int n, const oq_gate *g)
{
    if (oq_gate_check(g, n) != 0) return -1;
    oq_layout lay = {0, 0, UINT64_C(1) << n, 0};
    apply_local(g, psi, UINT64_C(1) << n, &lay);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Which chunks a gate touches (Sec. 3.3 index segments and control rules).  */
/* ------------------------------------------------------------------------- */
enum { OQ_JOB_NONE = 0, OQ_JOB_SINGLE = 1, OQ_JOB_PAIR_LO = 2, OQ_JOB_PAIR_HI = 3, OQ_JOB_PERMUTE_LO = 4, OQ_JOB_PERMUTE_HI = 5 };

static int is_unit(double re, double im) { return re == 1.0 && im == 0.0; }

/* Role of chunk c (global amplitudes c*2^cb ...) under gate g. */
int oq_chunk_role(const oq_gate *g, int cb, uint64_t c)
{
    uint64_t cm = g->control_mask;
    uint64_t cm_hi = cm >> cb;                       /* controls on chunk-index bits */
    uint64_t cm_lo = cm & ((UINT64_C(1) << cb) - 1); /* controls inside the chunk */
    if ((c & cm_hi) != cm_hi) return OQ_JOB_NONE;    /* a control bit is 0: chunk left unmodified */
    switch (g->kind) {
    case OQ_U1:
    case OQ_X:
        if ((int)g->target >= cb) {
            int hi = (int)((c >> (g->target - cb)) & 1u);
            if (g->kind == OQ_X && cm_lo == 0) return hi ? OQ_JOB_PERMUTE_HI : OQ_JOB_PERMUTE_LO;
            return hi ? OQ_JOB_PAIR_HI : OQ_JOB_PAIR_LO;
        }
        return OQ_JOB_SINGLE;
    case OQ_MCZ:
        return OQ_JOB_SINGLE;
    case OQ_DIAG1:
    case OQ_DIAG2: {
        /* touched unless every phase that can occur inside this chunk is 1 */
        int all_unit = 1;
        for (int idx = 0; idx < 4; ++idx) {
            if (g->kind == OQ_DIAG1 && idx >= 2) break;
            int b1 = idx & 1, b2 = idx >> 1;
            if ((int)g->target >= cb && (int)((c >> (g->target - cb)) & 1u) != b1) continue;
            if (g->kind == OQ_DIAG2 && (int)g->target2 >= cb && (int)((c >> (g->target2 - cb)) & 1u) != b2) continue;
            if (!is_unit(g->m[2 * idx], g->m[2 * idx + 1])) all_unit = 0;
        }
        return all_unit ? OQ_JOB_NONE : OQ_JOB_SINGLE;
    }
    default:
        return OQ_JOB_NONE;
    }
}

/* Sum of squares of C doubles, in index order. */
static double sum_sq(const double *x, int C)
{
    double a = 0.0;
    for (int i = 0; i < C; ++i) a += x[i] * x[i];
    return a;
}

/* One unit of the blockwise loop: decompress chunk c0 (and c1 for a pair
 * job), update its amplitudes, recompress each at its own level.  For a
 * single-chunk job pass in1 = NULL.  If n2 is not NULL, n2[k] receives the
 * squared norm of output chunk k after the update and before truncation, and
 * n2[2 + k] that of the values its new stream holds.  Returns 0 or -1. */
static int gate_job_n2(const oq_gate *g, int cb, int C, int flags,
                       uint64_t c0, const uint8_t *in0, size_t len0, int level0, uint8_t *out0, size_t *olen0,
                       uint64_t c1, const uint8_t *in1, size_t len1, int level1, uint8_t *out1, size_t *olen1,
                       double *n2)
{
    uint64_t ca = (uint64_t)C / 2;
    int two = in1 != NULL;
    /* a pair job exactly for U1 / X gates whose target indexes chunks */
    int pair_gate = (g->kind == OQ_U1 || g->kind == OQ_X) && (int)g->target >= cb;
    if (pair_gate != two || (two && (c1 ^ c0) != (UINT64_C(1) << (g->target - cb)))) return -1;
    double *psi = (double *)malloc(sizeof(double) * (size_t)C * (two ? 2 : 1));
    int rc = oq_decode_chunk(in0, len0, C, psi);
    if (rc == 0 && two) rc = oq_decode_chunk(in1, len1, C, psi + C);
    if (rc == 0) {
        oq_layout lay;
        lay.base0 = c0 << cb;
        lay.base1 = two ? (c1 << cb) : 0;
        lay.half = ca;
        lay.pair_units = two;
        apply_local(g, psi, two ? 2 * ca : ca, &lay);
        if (n2) {
            n2[0] = sum_sq(psi, C);
            n2[1] = two ? sum_sq(psi + C, C) : 0.0;
        }
        *olen0 = oq_encode_chunk_ex(psi, C, level0, flags, out0);
        if (two) *olen1 = oq_encode_chunk_ex(psi + C, C, level1, flags, out1);
        if (n2) {
            rc = oq_decode_chunk(out0, *olen0, C, psi);
            if (rc == 0 && two) rc = oq_decode_chunk(out1, *olen1, C, psi + C);
            n2[2] = sum_sq(psi, C);
            n2[3] = two ? sum_sq(psi + C, C) : 0.0;
        }
    }
    free(psi);
    return rc;
}

int oq_gate_job_ex(const oq_gate *g, int cb, int C, int flags,
                   uint64_t c0, const uint8_t *in0, size_t len0, int level0, uint8_t *out0, size_t *olen0,
                   uint64_t c1, const uint8_t *in1, size_t len1, int level1, uint8_t *out1, size_t *olen1)
{
    return gate_job_n2(g, cb, C, flags, c0, in0, len0, level0, out0, olen0, c1, in1, len1, level1, out1, olen1,
                       NULL);
}

int oq_gate_job(const oq_gate *g, int cb, int C,
                uint64_t c0, const uint8_t *in0, size_t len0, int level0, uint8_t *out0, size_t *olen0,
                uint64_t c1, const uint8_t *in1, size_t len1, int level1, uint8_t *out1, size_t *olen1)
{
    return oq_gate_job_ex(g, cb, C, 0, c0, in0, len0, level0, out0, olen0, c1, in1, len1, level1, out1, olen1);
}

/* ------------------------------------------------------------------------- */
/* Compressed simulator (Sec. 3.1, 3.3, 3.7, 3.8).                           */
/* ------------------------------------------------------------------------- */
enum { OQ_MODE_LOSSLESS = 0, OQ_MODE_FIXED = 1, OQ_MODE_ADAPTIVE = 2, OQ_MODE_PERBLOCK = 3 };

typedef struct {
    int n, cb, bl, C;
    uint64_t nchunks, nblocks;
    uint8_t **chunk;
    uint32_t *len;
    int mode, level;
    uint64_t budget;
    uint8_t *block_level;     /* used in per-block mode */
    double flb;               /* fidelity lower bound, Eq. (11) */
    double flb_weighted;      /* per-block mode: prod over gates of (1 - wd / nlb) */
    double norm2;             /* per-block mode: squared norm of the stored state */
    uint64_t gates_applied, lossy_steps;
    uint64_t min_compressed, max_compressed;
    int enc_flags;            /* OQ_ENC_ENTROPY: chunks may take the entropy-coded body;
                                 OQ_ENC_RESHUFFLE: Solution D value order */
    uint8_t *scratch_out[2];
} oq_sim;

static size_t pad4(size_t x) { return (x + 3) & ~(size_t)3; }

uint64_t oq_sim_compressed_bytes(const oq_sim *s)
{
    uint64_t tot = 0;
    for (uint64_t c = 0; c < s->nchunks; ++c) tot += pad4(s->len[c]);
    return tot;
}

/* State |0...0> stored in compressed form (Sec. 3.3: the state vectors are
 * created in blocks and compressed). */
oq_sim *oq_sim_create(int n, int block_log2, int mode, int fixed_level, uint64_t budget)
{
    if (n < 2 || n > 40 || block_log2 < 1 || block_log2 > n) return NULL;
    if (fixed_level < 0 || fixed_level >= OQ_NLEVELS) return NULL;
    oq_sim *s = (oq_sim *)calloc(1, sizeof(oq_sim));
    s->n = n;
    s->bl = block_log2;
    s->cb = block_log2 < 10 ? block_log2 : 10;
    s->C = 2 << s->cb;
    s->nchunks = UINT64_C(1) << (n - s->cb);
    s->nblocks = UINT64_C(1) << (n - s->bl);
    s->chunk = (uint8_t **)calloc(s->nchunks, sizeof(uint8_t *));
    s->len = (uint32_t *)calloc(s->nchunks, sizeof(uint32_t));
    s->mode = mode;
    s->level = (mode == OQ_MODE_FIXED) ? fixed_level : 0;
    s->budget = budget;
    s->block_level = (uint8_t *)calloc(s->nblocks, 1);
    if (mode == OQ_MODE_PERBLOCK) memset(s->block_level, fixed_level, s->nblocks);
    s->flb = 1.0;
    s->flb_weighted = 1.0;
    s->norm2 = 1.0;
    size_t cap = oq_chunk_cap(s->C);
    s->scratch_out[0] = (uint8_t *)malloc(cap);
    s->scratch_out[1] = (uint8_t *)malloc(cap);
    double *zero = (double *)calloc((size_t)s->C, sizeof(double));
    for (uint64_t c = 0; c < s->nchunks; ++c) {
        if (c == 0) zero[0] = 1.0;
        size_t L = oq_encode_chunk(zero, s->C, 0, s->scratch_out[0]);
        s->chunk[c] = (uint8_t *)malloc(L);
        memcpy(s->chunk[c], s->scratch_out[0], L);
        s->len[c] = (uint32_t)L;
        zero[0] = 0.0;
    }
    free(zero);
    s->min_compressed = s->max_compressed = oq_sim_compressed_bytes(s);
    return s;
}

void oq_sim_destroy(oq_sim *s)
{
    if (!s) return;
    for (uint64_t c = 0; c < s->nchunks; ++c) free(s->chunk[c]);
    free(s->chunk); free(s->len); free(s->block_level);
    free(s->scratch_out[0]); free(s->scratch_out[1]);
    free(s);
}

static int chunk_level(const oq_sim *s, uint64_t c)
{
    if (s->mode == OQ_MODE_PERBLOCK) return s->block_level[c >> (s->bl - s->cb)];
    return s->level;
}

/* Replacement record kept until the gate commits (so it can be undone). */
typedef struct { uint64_t c; uint8_t *old; uint32_t old_len; } oq_undo;

/* Apply gate g to the compressed state.  Old chunk versions are returned in
 * undo[] (count in *nundo) so the caller can commit or roll back.  Sets
 * *reencoded to the number of chunks recompressed, *wd to the sum over them
 * of delta(level of the chunk) * (squared norm of the chunk after the update,
 * before truncation) and *lost to the squared norm the truncation removed. */
static int sim_gate(oq_sim *s, const oq_gate *g, oq_undo *undo, uint64_t *nundo, uint64_t *reencoded, double *wd,
                    double *lost)
{
    *nundo = 0;
    *reencoded = 0;
    *wd = 0.0;
    *lost = 0.0;
    double n2[4];
    for (uint64_t c = 0; c < s->nchunks; ++c) {
        int role = oq_chunk_role(g, s->cb, c);
        if (role == OQ_JOB_NONE || role == OQ_JOB_PAIR_HI || role == OQ_JOB_PERMUTE_HI) continue;
        if (role == OQ_JOB_PERMUTE_LO) {
            /* X on chunk-index bits with no in-chunk control: exchange the
             * two compressed chunks without recompressing (exact). */
            uint64_t c1 = c | (UINT64_C(1) << (g->target - s->cb));
            uint8_t *tp = s->chunk[c]; s->chunk[c] = s->chunk[c1]; s->chunk[c1] = tp;
            uint32_t tl = s->len[c]; s->len[c] = s->len[c1]; s->len[c1] = tl;
            undo[(*nundo)++] = (oq_undo){c, NULL, 0};   /* NULL marks a swap record */
            continue;
        }
        size_t o0 = 0, o1 = 0;
        if (role == OQ_JOB_SINGLE) {
            if (gate_job_n2(g, s->cb, s->C, s->enc_flags, c, s->chunk[c], s->len[c], chunk_level(s, c),
                            s->scratch_out[0], &o0, 0, NULL, 0, 0, NULL, NULL, n2) != 0) return -1;
            *wd += oq_delta_tab[chunk_level(s, c)] * n2[0];
            *lost += n2[0] - n2[2];
            undo[(*nundo)++] = (oq_undo){c, s->chunk[c], s->len[c]};
            s->chunk[c] = (uint8_t *)malloc(o0);
            memcpy(s->chunk[c], s->scratch_out[0], o0);
            s->len[c] = (uint32_t)o0;
            *reencoded += 1;
        } else { /* OQ_JOB_PAIR_LO */
            uint64_t c1 = c | (UINT64_C(1) << (g->target - s->cb));
            if (gate_job_n2(g, s->cb, s->C, s->enc_flags, c, s->chunk[c], s->len[c], chunk_level(s, c),
                            s->scratch_out[0], &o0, c1, s->chunk[c1], s->len[c1], chunk_level(s, c1),
                            s->scratch_out[1], &o1, n2) != 0)
                return -1;
            *wd += oq_delta_tab[chunk_level(s, c)] * n2[0];
            *wd += oq_delta_tab[chunk_level(s, c1)] * n2[1];
            *lost += (n2[0] - n2[2]) + (n2[1] - n2[3]);
            undo[(*nundo)++] = (oq_undo){c, s->chunk[c], s->len[c]};
            undo[(*nundo)++] = (oq_undo){c1, s->chunk[c1], s->len[c1]};
            s->chunk[c] = (uint8_t *)malloc(o0);
            memcpy(s->chunk[c], s->scratch_out[0], o0);
            s->len[c] = (uint32_t)o0;
            s->chunk[c1] = (uint8_t *)malloc(o1);
            memcpy(s->chunk[c1], s->scratch_out[1], o1);
            s->len[c1] = (uint32_t)o1;
            *reencoded += 2;
        }
    }
    return 0;
}

static void sim_commit(oq_undo *undo, uint64_t nundo)
{
    for (uint64_t k = 0; k < nundo; ++k) free(undo[k].old);
}

static void sim_rollback(oq_sim *s, const oq_gate *g, oq_undo *undo, uint64_t nundo)
{
    for (uint64_t k = nundo; k-- > 0;) {
        uint64_t c = undo[k].c;
        if (undo[k].old == NULL) {
            uint64_t c1 = c | (UINT64_C(1) << (g->target - s->cb));
            uint8_t *tp = s->chunk[c]; s->chunk[c] = s->chunk[c1]; s->chunk[c1] = tp;
            uint32_t tl = s->len[c]; s->len[c] = s->len[c1]; s->len[c1] = tl;
        } else {
            free(s->chunk[c]);
            s->chunk[c] = undo[k].old;
            s->len[c] = undo[k].old_len;
        }
    }
}

/* Apply a gate list.  Returns the number of gates applied (all of them on
 * success); a negative value -(k+1) reports that gate k could not be fitted
 * into the budget even at the loosest level (-2 - k: malformed gate k). */
long oq_sim_apply(oq_sim *s, const oq_gate *gates, size_t ngates)
{
    uint64_t max_undo = s->nchunks;
    oq_undo *undo = (oq_undo *)malloc(sizeof(oq_undo) * (size_t)max_undo);
    for (size_t k = 0; k < ngates; ++k) {
        const oq_gate *g = &gates[k];
        if (oq_gate_check(g, s->n) != 0) { free(undo); return -2 - (long)k; }
        uint64_t nundo = 0, reenc = 0;
        double wd = 0.0, lost = 0.0;
        for (;;) {
            if (sim_gate(s, g, undo, &nundo, &reenc, &wd, &lost) != 0) { free(undo); return -2 - (long)k; }
            uint64_t cbytes = oq_sim_compressed_bytes(s);
            if (s->mode != OQ_MODE_ADAPTIVE || s->budget == 0 || cbytes <= s->budget) {
                sim_commit(undo, nundo);
                break;
            }
            /* Sec. 3.7: the compressed state does not fit -> relax the bound
             * to the next level and redo the gate from its input. */
            sim_rollback(s, g, undo, nundo);
            if (s->level >= OQ_NLEVELS - 1) { free(undo); return -1 - (long)k; }
            s->level += 1;
        }
        if (reenc > 0) {
            if (s->mode == OQ_MODE_PERBLOCK) {
                /* Sec. 3.8 with a bound that varies by chunk: truncating v at
                 * relative error delta_c per value keeps <v|T(v)> at least
                 * |v|^2 - wd, so the step fidelity is at least 1 - wd/|v|^2,
                 * and |v|^2 is the norm before the gate (unitary update). */
                if (wd > 0.0) {
                    s->flb_weighted *= (1.0 - wd / s->norm2);
                    s->lossy_steps += 1;
                }
                s->norm2 -= lost;
            } else if (s->level > 0) {
                s->flb *= (1.0 - oq_delta_tab[s->level]);   /* Eq. (11) */
                s->lossy_steps += 1;
            }
        }
        s->gates_applied += 1;
        uint64_t cb = oq_sim_compressed_bytes(s);
        if (cb < s->min_compressed) s->min_compressed = cb;
        if (cb > s->max_compressed) s->max_compressed = cb;
    }
    free(undo);
    return (long)ngates;
}

/* Decode the whole state into psi (2*2^n doubles). */
int oq_sim_read_all(const oq_sim *s, double *psi)
{
    for (uint64_t c = 0; c < s->nchunks; ++c)
        if (oq_decode_chunk(s->chunk[c], s->len[c], s->C, psi + c * (uint64_t)s->C) != 0) return -1;
    return 0;
}

/* Copy chunk c's bytes into out (capacity cap); returns its length or 0. */
size_t oq_sim_chunk(const oq_sim *s, uint64_t c, uint8_t *out, size_t cap)
{
    if (c >= s->nchunks || s->len[c] > cap) return 0;
    memcpy(out, s->chunk[c], s->len[c]);
    return s->len[c];
}

/* Replace chunk c by the given bytes (checkpoint reload / test setup). */
int oq_sim_set_chunk(oq_sim *s, uint64_t c, const uint8_t *in, size_t len)
{
    if (c >= s->nchunks || len > oq_chunk_cap(s->C)) return -1;
    double *psi = (double *)malloc(sizeof(double) * (size_t)s->C);
    int rc = oq_decode_chunk(in, len, s->C, psi);
    free(psi);
    if (rc != 0) return -1;
    free(s->chunk[c]);
    s->chunk[c] = (uint8_t *)malloc(len);
    memcpy(s->chunk[c], in, len);
    s->len[c] = (uint32_t)len;
    return 0;
}

/* Codec flags of later encodes (OQ_ENC_ENTROPY: the entropy-coded body is
 * taken when it is smaller).  The initial state is the same either way. */
void oq_sim_set_codec(oq_sim *s, int flags) { s->enc_flags = flags & (OQ_ENC_ENTROPY | OQ_ENC_RESHUFFLE); }

int oq_sim_set_block_level(oq_sim *s, uint64_t b, int level)
{
    if (b >= s->nblocks || level < 0 || level >= OQ_NLEVELS) return -1;
    s->block_level[b] = (uint8_t)level;
    return 0;
}

/* Footprint summary: out[0] compressed bytes (sum of 4-byte padded chunk
 * sizes), out[1] number of chunks, out[2] current level, out[3] gates
 * applied, out[4] lossy steps, out[5] min compressed bytes, out[6] max
 * compressed bytes; fout[0] fidelity lower bound (Eq. (11)), fout[1] the
 * per-block weighted bound. */
void oq_sim_footprint(const oq_sim *s, uint64_t *out, double *fout)
{
    out[0] = oq_sim_compressed_bytes(s);
    out[1] = s->nchunks;
    out[2] = (uint64_t)s->level;
    out[3] = s->gates_applied;
    out[4] = s->lossy_steps;
    out[5] = s->min_compressed;
    out[6] = s->max_compressed;
    fout[0] = s->flb;
    fout[1] = s->flb_weighted;
}

int oq_sim_chunk_log2(const oq_sim *s) { return s->cb; }

// Solution B of Sec. 4.2 on the GPU: each value is quantized in the
// logarithmic domain (the IEEE-754 bit pattern of |x| read as an integer, a
// piecewise-linear log2), predicted from the previous nonzero value of the
// same part (real parts from real parts, imaginary from imaginary), and the
// codes (16,384 symbols) are Huffman coded with canonical codes.  Stream
// layout, header mode 3:
//   u32 header | u16 symbols per code length 1..16 | u16 bit length of each
//   sub-stream of 32 symbols | u16 symbols in canonical order, padded to 4
//   bytes | codes, first bit first into an LSB-first bit stream, every code
//   but an escape's followed by the sign bit, padded to 4 bytes | u64 escaped
//   values in coding order.
// Coding order: real parts of the chunk's amplitudes, then imaginary parts.
// Bins: k = floor((v + W/2) / W), W = 2^w, w = 52 - t, t = 16, 13, 9, 6, 3
// for 1e-5 .. 1e-1 (the largest t with 2^-(t+1) <= epsilon); a value is
// rebuilt as k W with its sign.  Codes are quantized before they are
// predicted (k_j - k_p, p the previous nonzero value of the part), so every
// symbol depends on the input values alone and the positions are coded in
// parallel.  Symbols: 0 escape (first nonzero value of a part, a code outside
// [-8190, 8191], a subnormal, inf, NaN, or k W beyond the finite range),
// 1 zero, 2 + 8190 + code.  Huffman lengths: leaves in (count, symbol) order,
// two queues, the leaf first on equal weights; a lone symbol takes length 1;
// with at most 2048 values no length exceeds 16.
//
// One workgroup of 256 threads per chunk (grid-stride over chunks); a
// thread holds P = C / 256 consecutive positions of the coding order.
#include "qcz_internal.h"

namespace qcz {
namespace {

constexpr int kNT = 256;
constexpr int kPMax = kCMax / kNT;
constexpr int kSub = 32;
constexpr int kMaxLen = 16;
constexpr uint32_t kModePred = 3u;
constexpr int kBitWords = (kCMax * (kMaxLen + 1) + 31) / 32 + 2;
constexpr int kHeadHalves = 2 + 16 + kCMax / kSub + kCMax + 2;   // u16 slots of the header area

__device__ __forceinline__ int pred_w(int level)
{
    switch (level) {
    case 1: return 36;
    case 2: return 39;
    case 3: return 43;
    case 4: return 46;
    case 5: return 49;
    default: return -1;
    }
}

__device__ __forceinline__ uint64_t d2u_(double x) { return (uint64_t)__double_as_longlong(x); }
__device__ __forceinline__ double u2d_(uint64_t u) { return __longlong_as_double((long long)u); }

__device__ __forceinline__ int64_t qbin(uint64_t mag, int w) { return (int64_t)((mag + (1ull << (w - 1))) >> w); }

// workgroup exclusive prefix sum (256 threads, four wavefronts); sh: 4 words
__device__ uint32_t wg_exscan(uint32_t v, uint32_t *sh, uint32_t &total)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t x = v;
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) sh[wv] = x;
    __syncthreads();
    uint32_t off = 0, tot = 0;
    for (int i = 0; i < kNT / 64; ++i) {
        const uint32_t t = sh[i];
        off += i < wv ? t : 0u;
        tot += t;
    }
    __syncthreads();
    total = tot;
    return off + x - v;
}

// workgroup exclusive max scan of int32 (-1 below every value)
__device__ int wg_exmax(int v, int *sh)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int x = v;
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(x, d, 64);
        if (lane >= d) x = max(x, y);
    }
    int ex = __shfl_up(x, 1, 64);
    if (lane == 0) ex = -1;
    if (lane == 63) sh[wv] = x;
    __syncthreads();
    int off = -1;
    for (int i = 0; i < kNT / 64; ++i)
        if (i < wv) off = max(off, sh[i]);
    __syncthreads();
    return max(off, ex);
}

// workgroup segmented inclusive scan: (f, v) pairs, a set flag restarts the sum
__device__ void seg_combine(int &fa, int64_t &va, int fb, int64_t vb)
{
    va = fb ? vb : va + vb;
    fa = fa | fb;
}

__device__ void wg_segscan_ex(int f, int64_t v, int64_t *shv, int *shf, int &fout, int64_t &vout)
{
    // exclusive: the combination of every earlier thread's pair
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int fi = f;
    int64_t vi = v;
    for (int d = 1; d < 64; d <<= 1) {
        const int fy = __shfl_up(fi, d, 64);
        const int64_t vy = __shfl_up(vi, d, 64);
        if (lane >= d) {
            int fa = fy;
            int64_t va = vy;
            seg_combine(fa, va, fi, vi);
            fi = fa;
            vi = va;
        }
    }
    int fe = __shfl_up(fi, 1, 64);
    int64_t ve = __shfl_up(vi, 1, 64);
    if (lane == 0) { fe = 0; ve = 0; }
    if (lane == 63) { shf[wv] = fi; shv[wv] = vi; }
    __syncthreads();
    int fo = 0;
    int64_t vo = 0;
    for (int i = 0; i < kNT / 64; ++i)
        if (i < wv) seg_combine(fo, vo, shf[i], shv[i]);
    __syncthreads();
    seg_combine(fo, vo, fe, ve);
    fout = fo;
    vout = vo;
}

// bitonic sort of n (power of two, <= kCMax) u32 keys, ascending
__device__ void wg_sort(uint32_t *key, int n)
{
    for (int k = 2; k <= n; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int p = threadIdx.x; p < n / 2; p += kNT) {
                const int i = 2 * j * (p / j) + (p % j), ixj = i + j;
                const uint32_t a = key[i], b = key[ixj];
                const bool up = (i & k) == 0;
                if ((a > b) == up) { key[i] = b; key[ixj] = a; }
            }
            __syncthreads();
        }
}

__device__ int bsearch16(const uint16_t *a, int n, uint32_t v)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(kNT) void pred_encode_kernel(const double *in, int C, int level, uint64_t nchunks,
                                                          uint32_t *slots, uint64_t slot_words, uint32_t *sizes)
{
    __shared__ int32_t sk[kCMax];                 // bin of the magnitude per position (< 2^28: w >= 36)
    __shared__ uint16_t ssym[kCMax];              // symbol per position
    __shared__ uint32_t skey[kCMax];              // sort keys
    __shared__ uint32_t sw[kCMax];                // run starts, Huffman node weights, sub-stream starts
    __shared__ uint16_t spar[2 * kCMax];          // Huffman parents
    __shared__ uint16_t sdsym[kCMax];             // distinct symbols, increasing
    __shared__ uint32_t scode[kCMax];             // per distinct symbol: code | length << 16
    __shared__ uint8_t sdep[2 * kCMax];           // Huffman depths: leaves, then nodes
    __shared__ uint32_t sbits[kBitWords];
    __shared__ __align__(4) uint16_t shead[kHeadHalves];
    __shared__ uint32_t ssc[8];
    __shared__ int ssi[8];
    __shared__ uint32_t s_cntl[kMaxLen + 2], s_firstc[kMaxLen + 2], s_firsti[kMaxLen + 2];

    const int tid = threadIdx.x;
    const int w = pred_w(level);
    const int A = C / 2, P = C / kNT, NS = C / kSub;
    for (uint64_t chunk = blockIdx.x; chunk < nchunks; chunk += gridDim.x) {
        const double *x = in + chunk * (uint64_t)C;
        // 1. bins and zero flags of my positions
        uint64_t bits_[kPMax];
        int lastnz = -1;
#pragma unroll
        for (int i = 0; i < kPMax; ++i) {
            if (i >= P) break;
            const int j = tid * P + i, part = j >= A ? 1 : 0, a = part ? j - A : j;
            const uint64_t b = d2u_(x[2 * a + part]);
            bits_[i] = b;
            const uint64_t mag = b & 0x7FFFFFFFFFFFFFFFull;
            sk[j] = (int32_t)qbin(mag, w);
            if (mag != 0) lastnz = j;
        }
        // 2. previous nonzero position of the same part
        const int before = wg_exmax(lastnz, ssi);
        uint32_t nesc_mine = 0;
        {
            int prev = before;
#pragma unroll
            for (int i = 0; i < kPMax; ++i) {
                if (i >= P) break;
                const int j = tid * P + i, part = j >= A ? 1 : 0;
                const uint64_t b = bits_[i], mag = b & 0x7FFFFFFFFFFFFFFFull;
                const int p = (part && prev < A) ? -1 : prev;
                uint32_t sym;
                if (mag == 0) {
                    sym = 1u;
                } else {
                    const uint64_t e = mag >> 52;
                    const int64_t k = sk[j];   // (bins of inf and NaN too: below 2^28)
                    const uint64_t rb = (uint64_t)k << w;
                    const bool quant = e != 0 && e != 0x7FF && ((rb >> 52) & 0x7FF) != 0x7FF && (rb >> 63) == 0;
                    sym = 0u;
                    if (p >= 0 && quant) {
                        const int64_t d = k - (int64_t)sk[p];
                        if (d >= -8190 && d <= 8191) sym = (uint32_t)(2 + 8190 + d);
                    }
                    prev = j;
                }
                ssym[j] = (uint16_t)sym;
                skey[j] = sym;
                nesc_mine += sym == 0u ? 1u : 0u;
            }
        }
        __syncthreads();
        // 3. distinct symbols and their counts
        wg_sort(skey, C);
        uint32_t nb_mine = 0;
        for (int i = 0; i < P; ++i) {
            const int j = tid * P + i;
            nb_mine += (j == 0 || skey[j] != skey[j - 1]) ? 1u : 0u;
        }
        uint32_t nd = 0;
        uint32_t d0 = wg_exscan(nb_mine, ssc, nd);
        for (int i = 0; i < P; ++i) {
            const int j = tid * P + i;
            if (j == 0 || skey[j] != skey[j - 1]) {
                sdsym[d0] = (uint16_t)skey[j];
                sw[d0] = (uint32_t)j;
                ++d0;
            }
        }
        __syncthreads();
        // leaves keyed by (count, symbol): count = next run start - run start
        int np = 1;
        while (np < (int)nd) np <<= 1;
        for (int d = tid; d < np; d += kNT)
            skey[d] = d < (int)nd ? (((d + 1 < (int)nd ? sw[d + 1] : (uint32_t)C) - sw[d]) << 14) | sdsym[d]
                                  : 0xFFFFFFFFu;
        __syncthreads();
        wg_sort(skey, np);
        // 4. Huffman code lengths (one thread: two queues over the sorted leaves)
        if (tid == 0) {
            if (nd == 1) {
                sdep[0] = 1;   // the lone leaf takes length 1
            } else {
                // weights: leaves 0..nd-1 from the keys, nodes nd..2nd-2 in sw[0..nd-2]
                int nl = 0, nn = 0;
                const int nleaves = (int)nd, total = 2 * nleaves - 1;
                for (int made = nleaves; made < total; ++made) {
                    int pick[2];
                    uint32_t pw[2];
                    for (int q = 0; q < 2; ++q) {
                        const bool has_leaf = nl < nleaves, has_node = nn < made - nleaves;
                        const uint32_t lw = has_leaf ? (skey[nl] >> 14) : 0u;
                        const uint32_t nw = has_node ? sw[nn] : 0u;
                        const bool take_leaf = has_leaf && (!has_node || lw <= nw);
                        if (take_leaf) { pick[q] = nl; pw[q] = lw; ++nl; }
                        else { pick[q] = nleaves + nn; pw[q] = nw; ++nn; }
                    }
                    sw[made - nleaves] = pw[0] + pw[1];
                    spar[pick[0]] = (uint16_t)(made - nleaves);
                    spar[pick[1]] = (uint16_t)(made - nleaves);
                }
                // depths: the root (created last) first, every node before its children
                sdep[total - 1] = 0;
                for (int i = total - 2; i >= 0; --i) sdep[i] = (uint8_t)(sdep[nleaves + spar[i]] + 1);
            }
        }
        __syncthreads();
        // 5. canonical order (length, symbol) and codes
        for (int i = tid; i < np; i += kNT)
            skey[i] = i < (int)nd ? (((uint32_t)sdep[i] << 14) | (skey[i] & 0x3FFFu)) : 0xFFFFFFFFu;
        if (tid <= kMaxLen + 1) s_cntl[tid] = 0;
        __syncthreads();
        wg_sort(skey, np);
        for (int i = tid; i < (int)nd; i += kNT) atomicAdd(&s_cntl[min(skey[i] >> 14, (uint32_t)kMaxLen + 1)], 1u);
        __syncthreads();
        if (tid == 0) {
            uint32_t c = 0, idx = 0;
            for (int l = 1; l <= kMaxLen; ++l) {
                s_firstc[l] = c;
                s_firsti[l] = idx;
                c = (c + s_cntl[l]) << 1;
                idx += s_cntl[l];
            }
        }
        for (int i = tid; i < kHeadHalves; i += kNT) shead[i] = 0;
        __syncthreads();
        const int hsym = 2 + 16 + NS;   // first symbol slot (u16) of the header area
        for (int i = tid; i < (int)nd; i += kNT) {
            const uint32_t l = skey[i] >> 14, sy = skey[i] & 0x3FFFu;
            const uint32_t code = s_firstc[l] + ((uint32_t)i - s_firsti[l]);
            scode[bsearch16(sdsym, (int)nd, sy)] = code | (l << 16);
            shead[hsym + i] = (uint16_t)sy;
        }
        if (tid >= 1 && tid <= kMaxLen) shead[2 + tid - 1] = (uint16_t)s_cntl[tid];
        if (tid == 0) { shead[0] = (uint16_t)(kModePred | ((uint32_t)level << 2)); shead[1] = 0; }
        const int nbw_max = (C * (kMaxLen + 1) + 31) / 32;
        for (int i = tid; i < nbw_max + 1; i += kNT) sbits[i] = 0;
        __syncthreads();
        // 6. bit positions (the coding order, sub-streams back to back) and codes
        uint32_t nbits_mine = 0;
        uint32_t cl[kPMax];
#pragma unroll
        for (int i = 0; i < kPMax; ++i) {
            if (i >= P) break;
            const int j = tid * P + i;
            const uint32_t sy = ssym[j];
            cl[i] = scode[bsearch16(sdsym, (int)nd, sy)];
            nbits_mine += (cl[i] >> 16) + (sy != 0u ? 1u : 0u);
        }
        uint32_t total_bits = 0;
        uint32_t pos = wg_exscan(nbits_mine, ssc, total_bits);
        uint32_t esc_total = 0;
        uint32_t esc0 = wg_exscan(nesc_mine, ssc, esc_total);
        const int hwords = (2 * (2 + 16 + NS) + 2 * (int)nd + 3) / 4;
        const int bwords = (int)((total_bits + 31) / 32);
        const uint64_t size = 4ull * (uint64_t)(hwords + bwords) + 8ull * esc_total;
        const bool fits = size <= 4ull * slot_words;
        uint32_t *out = slots + chunk * slot_words;
#pragma unroll
        for (int i = 0; i < kPMax; ++i) {
            if (i >= P) break;
            const int j = tid * P + i;
            const uint32_t sy = ssym[j], l = cl[i] >> 16, code = cl[i] & 0xFFFFu;
            if (j % kSub == 0) sw[j / kSub] = pos;   // start of sub-stream j / 32
            uint32_t v = __brev(code) >> (32 - l);   // first code bit at the lowest position
            uint32_t nb = l;
            if (sy != 0u) { v |= (uint32_t)(bits_[i] >> 63) << l; nb += 1; }
            else if (fits) {
                const uint64_t wi = (uint64_t)(hwords + bwords) + 2ull * esc0;
                out[wi] = (uint32_t)bits_[i];
                out[wi + 1] = (uint32_t)(bits_[i] >> 32);
                ++esc0;
            }
            const uint32_t o = pos & 31u, wi = pos >> 5;
            atomicOr(&sbits[wi], v << o);
            if (o + nb > 32) atomicOr(&sbits[wi + 1], v >> (32 - o));
            pos += nb;
        }
        __syncthreads();
        for (int i = tid; i < NS; i += kNT)
            shead[2 + 16 + i] = (uint16_t)((i + 1 < NS ? sw[i + 1] : total_bits) - sw[i]);
        __syncthreads();
        if (fits) {
            const uint32_t *h32 = reinterpret_cast<const uint32_t *>(shead);
            for (int i = tid; i < hwords; i += kNT) out[i] = h32[i];
            for (int i = tid; i < bwords; i += kNT) out[hwords + i] = sbits[i];
        }
        if (tid == 0) sizes[chunk] = fits ? (uint32_t)size : 0u;
        __syncthreads();
    }
}

__global__ __launch_bounds__(kNT) void pred_decode_kernel(const uint32_t *slots, uint64_t slot_words,
                                                          const uint32_t *sizes, int C, uint64_t nchunks,
                                                          double *outv)
{
    __shared__ uint32_t sbits[kBitWords];
    __shared__ uint16_t stab[kCMax];
    __shared__ uint16_t ssym[kCMax];
    __shared__ uint8_t ssgn[kCMax];
    __shared__ uint32_t s_cnt[kMaxLen + 2], s_firstc[kMaxLen + 2], s_firsti[kMaxLen + 2], s_sub[kCMax / kSub + 1];
    __shared__ int s_ok, s_w, s_nsym, s_hwords, s_bwords;
    __shared__ uint32_t ssc[8];
    __shared__ int64_t sv64[8];
    __shared__ int sfl[8];

    const int tid = threadIdx.x;
    const int A = C / 2, P = C / kNT, NS = C / kSub;
    for (uint64_t chunk = blockIdx.x; chunk < nchunks; chunk += gridDim.x) {
        const uint32_t *in = slots + chunk * slot_words;
        const uint32_t size = sizes[chunk];
        const uint32_t nw = (uint32_t)min<uint64_t>((size + 3u) / 4u, slot_words);
        const uint32_t hdr = (size >= 4 && nw >= 1) ? in[0] : 0u;
        if ((hdr & 3u) != kModePred) continue;   // (uniform: every thread reads the same header)
        auto half = [&](int h) -> uint32_t {
            const uint32_t wi = (uint32_t)h >> 1;
            return wi < nw ? ((in[wi] >> (16 * (h & 1))) & 0xFFFFu) : 0u;
        };
        if (tid == 0) {
            const int level = (int)((hdr >> 2) & 7u);
            int ok = (hdr >> 5) == 0 && pred_w(level) > 0 && size >= 4u * (uint32_t)(9 + NS / 2);
            uint32_t nsym = 0, kraft = 0;
            for (int l = 1; l <= kMaxLen; ++l) {
                s_cnt[l] = half(2 + l - 1);
                nsym += s_cnt[l];
                kraft += s_cnt[l] << (kMaxLen - l);
            }
            ok = ok && nsym >= 1 && nsym <= (uint32_t)C && kraft <= (1u << kMaxLen);
            uint32_t c = 0, idx = 0, tot = 0;
            for (int l = 1; l <= kMaxLen; ++l) {
                s_firstc[l] = c;
                s_firsti[l] = idx;
                c = (c + s_cnt[l]) << 1;
                idx += s_cnt[l];
            }
            for (int i = 0; i < NS; ++i) {
                s_sub[i] = tot;
                tot += half(2 + 16 + i);
            }
            s_sub[NS] = tot;
            s_hwords = (2 * (2 + 16 + NS) + 2 * (int)nsym + 3) / 4;
            s_bwords = (int)((tot + 31) / 32);
            ok = ok && (uint32_t)(s_hwords + s_bwords) <= nw && tot <= (uint32_t)(C * (kMaxLen + 1));
            s_ok = ok;
            s_w = pred_w(level);
            s_nsym = ok ? (int)nsym : 0;
        }
        __syncthreads();
        const int w = s_w;
        const bool ok = s_ok != 0;
        for (int i = tid; i < s_nsym; i += kNT) stab[i] = (uint16_t)min(half(2 + 16 + NS + i), 16383u);
        for (int i = tid; i < (ok ? s_bwords : 0); i += kNT) sbits[i] = in[s_hwords + i];
        if (ok && tid == 0) sbits[s_bwords] = 0;
        __syncthreads();
        // 1. symbols: one thread per sub-stream
        int bad = 0;
        if (ok && tid < NS) {
            uint32_t p = s_sub[tid];
            const uint32_t end = s_sub[tid + 1];
            for (int j = tid * kSub; j < (tid + 1) * kSub; ++j) {
                uint32_t v = 0, sy = 0xFFFFu;
                for (int l = 1; l <= kMaxLen && p < end; ++l) {
                    v = (v << 1) | ((sbits[p >> 5] >> (p & 31u)) & 1u);
                    ++p;
                    if (s_cnt[l] && v >= s_firstc[l] && v - s_firstc[l] < s_cnt[l]) {
                        sy = stab[s_firsti[l] + (v - s_firstc[l])];
                        break;
                    }
                }
                uint8_t sg = 0;
                if (sy == 0xFFFFu) { bad = 1; sy = 1u; }
                else if (sy != 0u) {
                    if (p < end) { sg = (uint8_t)((sbits[p >> 5] >> (p & 31u)) & 1u); ++p; }
                    else bad = 1;
                }
                ssym[j] = (uint16_t)sy;
                ssgn[j] = sg;
            }
            bad |= p != end ? 1 : 0;
        }
        (void)bad;
        __syncthreads();
        // 2. escapes in coding order, and the quantized magnitudes by a
        //    segmented sum over each part (an escape restarts it)
        uint32_t ne = 0;
        int fl[kPMax];
        int64_t val[kPMax];
        uint64_t escb[kPMax];
#pragma unroll
        for (int i = 0; i < kPMax; ++i) {
            if (i >= P) break;
            ne += (ok && ssym[tid * P + i] == 0u) ? 1u : 0u;
        }
        uint32_t ne_tot = 0;
        uint32_t e0 = wg_exscan(ne, ssc, ne_tot);
        int ft = 0;
        int64_t vt = 0;
#pragma unroll
        for (int i = 0; i < kPMax; ++i) {
            if (i >= P) break;
            const int j = tid * P + i;
            const uint32_t sy = ok ? ssym[j] : 1u;
            fl[i] = 0;
            val[i] = 0;
            escb[i] = 0;
            if (sy == 0u) {
                const uint64_t wi = (uint64_t)(s_hwords + s_bwords) + 2ull * e0;
                const uint64_t lo = wi < nw ? in[wi] : 0u, hi = wi + 1 < nw ? in[wi + 1] : 0u;
                escb[i] = lo | (hi << 32);
                fl[i] = 1;
                val[i] = qbin(escb[i] & 0x7FFFFFFFFFFFFFFFull, w > 0 ? w : 36);
                ++e0;
            } else if (sy >= 2u) {
                val[i] = (int64_t)sy - 2 - 8190;
            }
            seg_combine(ft, vt, fl[i], val[i]);
        }
        int fx = 0;
        int64_t vx = 0;
        wg_segscan_ex(ft, vt, sv64, sfl, fx, vx);
#pragma unroll
        for (int i = 0; i < kPMax; ++i) {
            if (i >= P) break;
            const int j = tid * P + i, part = j >= A ? 1 : 0, a = part ? j - A : j;
            seg_combine(fx, vx, fl[i], val[i]);
            const uint32_t sy = ok ? ssym[j] : 1u;
            uint64_t b;
            if (sy == 1u) b = (uint64_t)(ok ? ssgn[j] : 0u) << 63;
            else if (sy == 0u) b = escb[i];
            else b = ((uint64_t)vx << (w > 0 ? w : 36)) | ((uint64_t)ssgn[j] << 63);
            outv[chunk * (uint64_t)C + 2 * a + part] = u2d_(b);
        }
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_pred_encode(const double *in, int C, int level, uint64_t nchunks, uint32_t *slots,
                              uint64_t slot_words, uint32_t *sizes, hipStream_t st)
{
    if (C < kNT || C > kCMax || (C & (C - 1)) || level < 1 || level >= kLevels) return hipErrorInvalidValue;
    const int grid = (int)std::min<uint64_t>(nchunks, 4096);
    hipLaunchKernelGGL(pred_encode_kernel, dim3(grid), dim3(kNT), 0, st, in, C, level, nchunks, slots, slot_words,
                       sizes);
    return hipGetLastError();
}

hipError_t launch_pred_decode(const uint32_t *slots, uint64_t slot_words, const uint32_t *sizes, int C,
                              uint64_t nchunks, double *out, hipStream_t st)
{
    if (C < kNT || C > kCMax || (C & (C - 1))) return hipErrorInvalidValue;
    const int grid = (int)std::min<uint64_t>(nchunks, 4096);
    hipLaunchKernelGGL(pred_decode_kernel, dim3(grid), dim3(kNT), 0, st, slots, slot_words, sizes, C, nchunks, out);
    return hipGetLastError();
}

size_t pred_cap_bytes(int C)
{
    return 4 + 32 + 2 * (size_t)(C / kSub) + (((size_t)2 * C + 3) & ~(size_t)3) +
           4 * (size_t)((C * (kMaxLen + 1) + 31) / 32) + 8 * (size_t)C;
}

}  // namespace qcz

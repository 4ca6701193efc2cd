// Internal types shared by the HIP kernels (qcz_kernels.hip) and the host
// runtime (qcz_runtime.cpp) of the compressed state-vector library.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace qcz {

constexpr int kLevels = 6;          // lossless, 1e-5, 1e-4, 1e-3, 1e-2, 1e-1 (Sec. 3.7)
constexpr int kWG = 256;            // threads per workgroup: two chunk slots of 128
constexpr int kGroup = 128;         // threads per chunk slot
constexpr int kCMax = 2048;         // doubles per chunk (1024 amplitudes)
constexpr int kCMin = 128;          // one value per thread at least
constexpr int kBufWords = 4352;     // per-slot LDS words: kCMax doubles at padded positions
                                    // (one pad double per 16), or the largest stream plus the
                                    // slack its bit reader may touch
constexpr int kMaxBatch = 512;      // gates per launch batch (per-gate log entries)
constexpr int kStripes = 32;        // independent arena allocators (one cache line each)
constexpr int kMaxGrid = 8192;      // workgroups per gate launch
constexpr uint32_t kMaxChunkBytes = 4 + 4 * (kCMax / 16) + 8 * kCMax;   // 16900

enum GateKind { K_U1 = 0, K_DIAG1 = 1, K_DIAG2 = 2, K_X = 3, K_MCZ = 4 };
enum JobType { J_SINGLE = 0, J_PAIR = 1, J_PERMUTE = 2, J_GROUP = 3 };
enum StopReason { STOP_NONE = 0, STOP_BUDGET = 1, STOP_ARENA = 2, STOP_CORRUPT = 3 };
enum ChunkMode { M_PACK = 0, M_CONST2 = 1, M_SPARSE = 2 };

// One gate, lowered to a job enumeration over chunk indices.
struct GateDesc {
    int32_t kind, q, q2, seq;       // seq: position in the launch batch
    uint64_t cm;                    // control mask over amplitude-index bits
    double m[8];
    int32_t job_type;               // JobType
    int32_t nchunk_bits;            // log2(number of chunks)
    uint64_t fixed_mask, fixed_val; // chunk-index bits held fixed by the enumeration
    uint64_t pair_bit;              // PAIR / PERMUTE: chunk-index bit flipped by the target
    uint64_t nitems;                // enumerated chunk positions
    uint64_t njobs;                 // workgroup jobs (two positions each)
    int32_t check_phase;            // DIAG: skip chunks whose reachable phases are all 1
    int32_t per_block;              // level from the per-block table instead of the global one
    int32_t block_shift;            // log2(chunks per block)
    int32_t fixed_level;            // >= 0: codec kernels encode at this level
    uint64_t job0, job_end;         // jobs [job0, job_end) of this launch (job_end 0: all njobs)
    int32_t entropy;                // the encoder may take the entropy-coded body (header bit 5); its
                                    // kernels decode such streams too (C = 2048, two wavefronts per chunk)
    int32_t sweep;                  // every chunk is enumerated and lands in the other arena (DevPtrs::out):
                                    // chunks the gate leaves unchanged are copied there as they are
    uint64_t act_mask, act_val;     // a sweep acts on chunk c only if (c & act_mask) == act_val (the
                                    // control bits its plain enumeration would have held fixed)
    int32_t reshuffle;              // the encoder stores PACK / SPARSE values re parts first (header bit 6)
    int32_t pad_;
    uint64_t pair_bit2;             // GROUP: the second chunk-index bit of the groups
    uint64_t pair_bit3;             // GROUP: the third chunk-index bit (eight-chunk groups), or 0
};

// the jobs one launch of a gate runs, and the enumerated chunk positions per job
__host__ __device__ inline uint64_t items_per_job(const GateDesc &d)
{
    return d.job_type == J_GROUP ? (d.pair_bit3 ? 8 : 4) : 2;
}
__host__ __device__ inline uint64_t job_begin(const GateDesc &d) { return d.job_end ? d.job0 : 0; }
__host__ __device__ inline uint64_t job_stop(const GateDesc &d) { return d.job_end ? d.job_end : d.njobs; }

struct GateLog {
    uint64_t live;   // compressed bytes after the gate
    uint64_t bump;   // arena bytes used after the gate
    uint64_t reenc;  // chunks re-encoded by the gate
    uint64_t rd;     // padded stream bytes read by those jobs
    uint64_t wr;     // padded stream bytes written
    double wd;       // per-block levels: sum over re-encoded chunks of delta(level) * |chunk before truncation|^2
    double lost;     // per-block levels: squared norm removed by the truncation
    uint64_t hits;   // block cache: chunks whose new stream was copied from an identical job's
};

// Device-resident control block (first bytes of the pool).  The arena is
// [0, base) compacted streams, then kStripes stripes of stripe_size bytes,
// each filled by its own bump counter so that concurrent allocations from
// different workgroups do not contend for one address.
struct DevState {
    uint64_t base;        // start of the stripes
    uint64_t stripe_size; // bytes per stripe
    uint64_t nstripes;    // stripes in use (1 .. kStripes)
    uint64_t live;        // sum over chunks of the 4-byte padded size
    uint64_t arena_cap;   // bytes in one arena
    uint64_t budget;      // compressed-byte limit checked after each gate (0: none)
    int32_t level;        // global level used by gates
    int32_t stop;         // set by a gate epilogue: every later gate of the batch is skipped
    int32_t stop_reason;
    int32_t stop_seq;
    int32_t fail;         // an allocation of the current gate did not fit
    int32_t corrupt;      // a chunk entry pointed outside the arena
    uint32_t done;        // finished workgroups of the running kernel
    uint32_t pad0;
    uint64_t pad1[7];
    // -- below: not rewritten by the host header update --
    uint64_t stripe[kStripes][16];   // bytes used per stripe (first word of a 128-byte line)
    GateLog log[kMaxBatch];
};

// per-workgroup partial sums of a gate launch (no same-address atomics)
struct WgPart {
    uint64_t delta, reenc, rd, wr;
    double wd, lost;
    uint64_t hits;
};

// Pointers of one state, passed by value to every kernel.
struct DevPtrs {
    uint32_t *arena;            // current arena, word addressed
    uint32_t *out;              // where gate kernels write new streams: the current arena, or the
                                // other one for a sweep
    uint64_t arena_words;
    uint64_t *table;            // per chunk: (offset in words << 16) | size in bytes
    uint64_t *undo;             // per enumerated position: previous table entry
    const uint8_t *block_level; // per block
    DevState *ds;
    WgPart *wgp;                // [kMaxGrid]
    int32_t cb;                 // log2 amplitudes per chunk
    int32_t C;                  // doubles per chunk
    uint64_t nchunks;
};

// Inputs / outputs of the codec-only and readout kernels.
struct IOPtrs {
    const double *raw_in;       // [nitems][C] doubles
    double *raw_out;            // [nitems][C] doubles
    const uint32_t *slots_in;   // [nitems][slot_words] streams
    const uint32_t *sizes_in;   // [nitems] bytes
    uint32_t *slots_out;
    uint32_t *sizes_out;
    uint64_t slot_words;
    const uint64_t *list;       // readout: chunk ids (nullptr: positions are chunk ids + first)
    uint64_t first;
    double *partials;           // moments: [gridDim.x][4]
    double *cstats;             // chunk statistics: [chunk][kChunkStats]
    uint64_t *lsizes;           // per-level sizes: [block][kLevels] padded bytes (accumulated)
    const uint32_t *role;       // block cache, per job of the launch: 0 leader, else 1 + key slot
    const uint32_t *owner;      // block cache, per key slot: the leader job
    const WgPart *cparts;       // block cache: per-workgroup sums of the followers' copy kernel
    const GateDesc *run;        // fused run: the gates applied in one decode / encode pass
    int32_t nrun;
};

// Gate-layer fusion: at most this many gates per fused pass.
constexpr int kMaxRun = 64;

// Compressed block cache of one gate launch (Sec. 3.4, on the GPU): every job
// is keyed by a hash of its input streams and of the chunk-index bits the gate
// reads.  The first job to insert a key leads and is computed; the others
// follow: after an exact comparison of their streams with the leader's they
// copy its output, or compute when the bytes differ.
constexpr uint64_t kEmptyKey = ~0ull;
constexpr uint32_t kRoleDone = ~0u;   // a follower copied by the copy kernel
constexpr int kCopyGrid = 1024;       // workgroups of the followers' copy kernel
struct CachePtrs {
    uint64_t *keys;       // [tsize], kEmptyKey when free
    uint32_t *owner;      // [tsize]
    uint32_t *role;       // [jobs of the launch]
    uint64_t *jkey;       // [jobs of the launch] key of each job (kEmptyKey: leads without a match)
    WgPart *parts;        // [kCopyGrid] per-workgroup sums of the copy kernel
    uint64_t tsize;       // power of two, at least twice the jobs of the launch
    uint64_t key_mask;    // bits of the key kept (all but in tests that force collisions)
};

// Per-chunk statistics record (doubles): sum of squares, nonzero values, sum /
// max / min of their biased exponents, values whose top 8 / 16 / 24 bits equal
// the previous value's, sign changes, stored as two constants, padded bytes.
constexpr int kChunkStats = 12;
enum { CS_N2 = 0, CS_NZ, CS_ESUM, CS_EMAX, CS_EMIN, CS_EQ8, CS_EQ16, CS_EQ24, CS_SGN, CS_CONST2, CS_BYTES };

// Selector network 16 -> 64 -> 64 -> 6 (float parameters, packed W1 b1 W2 b2 W3 b3).
constexpr int kNIn = 16, kNH = 64, kNOut = 6;
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kNH * kNIn, kOffW2 = kOffB1 + kNH, kOffB2 = kOffW2 + kNH * kNH,
              kOffW3 = kOffB2 + kNH, kOffB3 = kOffW3 + kNOut * kNH, kNParams = kOffB3 + kNOut;   // 5638

inline uint32_t chunk_cap_bytes(int C) { return 4u + 4u * (uint32_t)((C + 15) / 16) + 8u * (uint32_t)C; }

// Arena bytes a stream of `size` bytes occupies: whole 16-byte units, so that
// every stream starts 16-byte aligned and moves in 16-byte loads and stores
// (the compressed-size ledger counts 4-byte padded sizes).
__host__ __device__ inline uint32_t alloc_bytes(uint32_t size) { return (size + 15u) & ~15u; }

// Host launchers (qcz_kernels.hip).
hipError_t launch_gate(const GateDesc &gd, const DevPtrs &P, int grid, hipStream_t st, int wpg,
                       hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);
// block cache: key the jobs (hash pass, which also clears the key table, then
// a dedupe pass), run the leaders
// (list 1, no gate epilogue), copy the followers whose inputs match (one
// wavefront per job), then run the remaining followers (list 2, closes the
// gate); both job launches with the same grid, at most kMaxGrid / 2
hipError_t launch_cache_plan(const GateDesc &gd, const DevPtrs &P, const CachePtrs &cp, hipStream_t st);
hipError_t launch_cache_copy(const GateDesc &gd, const DevPtrs &P, const CachePtrs &cp, hipStream_t st);
// a run of nrun in-chunk gates (device array `run`) in one pass over every
// chunk; gd: the run's first gate (its enumeration and batch position)
hipError_t launch_gate_run(const GateDesc &gd, const DevPtrs &P, const GateDesc *run, int nrun, int grid,
                           hipStream_t st, hipEvent_t t0, hipEvent_t t1);
hipError_t launch_gate_list(const GateDesc &gd, const DevPtrs &P, const CachePtrs &cp, int list, int grid,
                            hipStream_t st);
// a run of nrun chunk-pair gates on the two chunk-index bits of gd (J_GROUP:
// pair_bit, pair_bit2) in one pass over groups of four chunks (C = 2048)
hipError_t launch_group_run(const GateDesc &gd, const DevPtrs &P, const GateDesc *run, int nrun, int grid,
                            hipStream_t st, hipEvent_t t0, hipEvent_t t1);
hipError_t launch_permute(const GateDesc &gd, const DevPtrs &P, int grid, hipStream_t st);
hipError_t launch_rollback(const GateDesc &gd, const DevPtrs &P, int grid, hipStream_t st);
hipError_t launch_encode_raw(const GateDesc &gd, const DevPtrs &P, const IOPtrs &io, int grid, hipStream_t st);
hipError_t launch_decode_slots(const GateDesc &gd, const DevPtrs &P, const IOPtrs &io, int grid, hipStream_t st);
hipError_t launch_readout(const GateDesc &gd, const DevPtrs &P, const IOPtrs &io, int grid, hipStream_t st);
hipError_t launch_moments(const GateDesc &gd, const DevPtrs &P, const IOPtrs &io, int grid, hipStream_t st);
hipError_t launch_chunk_stats(const GateDesc &gd, const DevPtrs &P, const IOPtrs &io, int grid, hipStream_t st);
hipError_t launch_level_sizes(const GateDesc &gd, const DevPtrs &P, const IOPtrs &io, int grid, hipStream_t st);
hipError_t launch_zero_u64(uint64_t *p, uint64_t n, hipStream_t st);
hipError_t launch_dot(const double *a, const double *b, uint64_t npairs, double *partials, int grid, hipStream_t st);

// Selector kernels (qcz_select.hip).
struct FeatCtx {
    double f12, f13, f14, f15;   // context features shared by all blocks
    int32_t cpb;                 // chunks per block
    int32_t block_log2;
    uint64_t nblocks;
};
hipError_t launch_block_features(const double *cstats, const uint8_t *block_level, const FeatCtx &ctx, uint64_t nb,
                                 float *X, double *n2, hipStream_t st);
hipError_t launch_mlp_forward(const float *params, const float *X, uint64_t N, float *probs, uint8_t *argmax,
                              hipStream_t st);
size_t mlp_workspace_bytes(uint64_t N);
// the no-allocation training step: samples its static workspace holds, and the
// device address / size of this GPU's copy of it
constexpr uint64_t kMlpStaticSamples = 8192;
hipError_t mlp_static_workspace(void **out, size_t *bytes);
hipError_t launch_mlp_train(float *params, float *m, float *v, const float *X, const uint8_t *labels, uint64_t N,
                            float lr, uint32_t step, float *grad_out, float *loss_out, void *work, hipStream_t st);
hipError_t launch_fill_table(const DevPtrs &P, uint64_t entry0, uint64_t entry_rest, hipStream_t st);

// Solution B codec (qcz_pred.hip): C = 256 .. 2048, lossy levels; encoded
// sizes above the slot are reported as 0; the decoder writes only the
// chunks whose header has mode 3 (the job kernel's slot decoder skips them)
hipError_t launch_pred_encode(const double *in, int C, int level, uint64_t nchunks, uint32_t *slots,
                              uint64_t slot_words, uint32_t *sizes, hipStream_t st);
hipError_t launch_pred_decode(const uint32_t *slots, uint64_t slot_words, const uint32_t *sizes, int C,
                              uint64_t nchunks, double *out, hipStream_t st);
size_t pred_cap_bytes(int C);
hipError_t launch_compact(const DevPtrs &P, uint32_t *dst_arena, uint64_t *scratch, uint64_t *block_sums,
                          uint64_t nblocks_scan, hipStream_t st);

}  // namespace qcz

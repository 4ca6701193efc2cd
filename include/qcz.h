/*
 * qcz.h -- C ABI of the MI355X compressed full-state quantum circuit
 * simulator (Wu et al., "Full-State Quantum Circuit Simulation by Using Data
 * Compression", SC'19).
 *
 * A 2^n-amplitude complex128 state is held as independently compressed
 * chunks in device memory.  Each gate decompresses the chunks it touches,
 * applies its 2x2 unitary to the amplitude pairs (Sec. 3.1, Eqs. (6), (7)),
 * and recompresses them with the hybrid lossless / error-bounded lossy scheme
 * of Sec. 3.7 and Sec. 4.2 (Solution C: truncation to Sig_Bit_Count bits,
 * Eq. (12), and the XOR leading-byte code), under the per-timestep adaptive
 * bound of Sec. 3.7.
 *
 * Conventions shared by every call:
 *   - qubit k is bit k of the amplitude index (Sec. 2.1, Eq. (5));
 *   - amplitudes are stored as interleaved doubles (re, im);
 *   - a "chunk" holds C = min(2048, 2b) doubles (min(1024, b) amplitudes) and
 *     is the unit of compression; a "block" of b = 2^block_log2 amplitudes
 *     groups chunks and carries an error level in the per-block mode;
 *   - error levels: 0 lossless, 1..5 the pointwise relative bounds
 *     1e-5, 1e-4, 1e-3, 1e-2, 1e-1 (Sec. 3.7);
 *   - all device work is queued on the stream given to qcz_create; calls
 *     that return host data synchronize that stream;
 *   - the caller owns every buffer it passes; the library keeps no pointer
 *     to caller memory except the device pool given to qcz_create, which
 *     must stay allocated until qcz_destroy;
 *   - no call throws; each returns a qcz_status and qcz_last_error() gives
 *     the message of the last failure on a state.
 */
#ifndef QCZ_H
#define QCZ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qcz_state qcz_state;

typedef enum {
    QCZ_OK = 0,
    QCZ_E_INVAL = -1,   /* malformed argument or gate record */
    QCZ_E_NOMEM = -2,   /* the state does not fit the budget at the loosest level, or the pool is too small */
    QCZ_E_DEVICE = -3,  /* a HIP call failed */
    QCZ_E_FORMAT = -4,  /* a compressed stream or chunk entry is malformed */
    QCZ_E_STATE = -5    /* call not allowed in the current state */
} qcz_status;

typedef enum {
    QCZ_MODE_LOSSLESS = 0,  /* every chunk lossless (level 0) */
    QCZ_MODE_FIXED = 1,     /* every gate at config.level */
    QCZ_MODE_ADAPTIVE = 2,  /* Sec. 3.7: start lossless, relax one level whenever the
                               compressed state exceeds budget_bytes after a gate, and
                               redo that gate from its input */
    QCZ_MODE_PERBLOCK = 3   /* level per block, set by qcz_set_block_levels */
} qcz_mode;

/* flags */
#define QCZ_FLAG_GRAPH 1u   /* replay launch batches from captured HIP graphs when a batch repeats */
#define QCZ_FLAG_TIMING 2u  /* time every fused gate kernel with HIP events on the state's stream
                               (launches directly, so it takes precedence over QCZ_FLAG_GRAPH) */
#define QCZ_FLAG_AUTOTUNE 4u /* over the first launch batches, rotate the fused kernel's launch shape
                                (wavefronts per chunk x workgroups per CU), time each shape with events and
                                keep the fastest per recompressed chunk; results do not depend on the shape */
#define QCZ_FLAG_RANGES 8u  /* modes without a size budget: a gate whose new streams do not fit beside the
                               live ones even after compaction, nor as a sweep into the other arena (a gate
                               that does not fit beside the live streams is first tried as one launch writing
                               every chunk into the other, empty arena; that needs no flag and keeps the
                               state at the last committed gate when it stops), runs in job ranges, each committed before the
                               next, so the arena only needs the live state plus one range.  The price: a
                               gate that still runs out of arena midway cannot be undone (its replaced
                               streams are gone); the call returns QCZ_E_NOMEM and the state is invalid
                               (later qcz_apply_gates calls return QCZ_E_STATE).  Without the flag such a
                               gate fails with QCZ_E_NOMEM and the state stays at the previous gate. */
#define QCZ_FLAG_CACHE 16u  /* compressed block cache (Sec. 3.4), per gate: jobs whose input streams and
                               gate action equal another job's (byte-exact comparison after a hash match)
                               copy that job's new streams instead of decompressing, applying and
                               recompressing.  Results are identical with or without it.  Gates over
                               per-block levels (QCZ_MODE_PERBLOCK) and gates run in job ranges do not use
                               it; after 32 cached gates in a row without a hit it switches itself off.
                               Needs a larger pool (qcz_pool_bytes_min); not with QCZ_FLAG_AUTOTUNE. */
#define QCZ_FLAG_CACHE_COLLIDE 32u /* test hook: keep 3 bits of the cache keys, so that different
                                      streams share keys and only the byte comparison separates them */
#define QCZ_FLAG_FUSE 64u   /* gate-layer fusion, QCZ_MODE_FIXED / QCZ_MODE_LOSSLESS: consecutive gates whose
                               jobs lie inside single chunks (targets on in-chunk qubits, diagonal gates and
                               multi-controlled Z on any qubits, any controls) run as one pass per batch run
                               (up to 64 gates): one decode of every chunk; each chunk takes, in order, the
                               gates that touch it, each followed by the truncation its re-encoding would
                               apply (Sec. 3.7; none for a chunk holding a subnormal value); one encode of the
                               chunks some gate touched.  Bytes and ledger equal the gate-by-gate run's; each
                               gate of a run counts the run's re-encoded chunks, the stream bytes moved are
                               counted once per pass, and min / max compressed bytes are sampled after each
                               pass.  Direct launches only (not inside replayed graphs); not with
                               QCZ_FLAG_AUTOTUNE; gates of the block cache are not fused. */

#define QCZ_FLAG_ENTROPY 128u /* the entropy-coding stage (Sec. 4.2: Solution C's lossless stage ends in an
                               entropy coder): a PACK or SPARSE chunk may carry its residuals in 4-bit lanes,
                               each stored raw, as one constant or by a canonical Huffman code of at most 8
                               bits, in sub-streams of 16 positions (header bit 5), whenever that is smaller.
                               Lossless: decoded values are those of the run without it.  Needs
                               block_log2 >= 10 (2048-double chunks) and two wavefronts per chunk; not with
                               QCZ_FLAG_CACHE or QCZ_FLAG_AUTOTUNE. */
#define QCZ_FLAG_GROUPS 512u /* with QCZ_FLAG_FUSE: consecutive U1 / X gates whose targets are chunk-index qubits
                               (chunk-pair jobs, any controls) on at most three distinct target bits (two when
                               the state has only two chunk-index bits) run as one pass over groups of the
                               eight (four) chunks those bits join (up to 64 gates): each chunk decoded and
                               encoded once, each gate followed by the truncation its re-encoding would apply
                               to the chunks it touched.  Same bytes and ledger as gate by gate.  2048-double
                               chunks, not with QCZ_FLAG_ENTROPY.  The pass holds its chunks in LDS (one or two
                               workgroups per CU instead of three), so it pays where pair passes dominate;
                               measure before enabling. */
#define QCZ_FLAG_RESHUFFLE 256u /* Solution D (Sec. 4.2): PACK and SPARSE chunks store their values re parts
                               first, then im parts (header bit 6), before the Solution C steps; decoded
                               values are those of the run without it.  Chunks created by qcz_create are
                               interleaved; every kernel decodes both orders. */

typedef struct {
    uint32_t n_qubits;      /* 6 .. 40 */
    uint32_t block_log2;    /* log2 amplitudes per block, 6 .. n_qubits */
    int32_t mode;           /* qcz_mode */
    int32_t level;          /* QCZ_MODE_FIXED: the level; QCZ_MODE_PERBLOCK: the initial level */
    uint64_t budget_bytes;  /* QCZ_MODE_ADAPTIVE: limit on compressed bytes (0: none) */
    uint32_t flags;         /* QCZ_FLAG_* */
    uint32_t batch;         /* gates per launch batch between host checks (0: 64; at most 512) */
    uint32_t grid;          /* workgroups per gate launch (0: 3 per compute unit) */
    uint32_t chunk_waves;   /* wavefronts working on one chunk in the gate kernel: 2, 4 or 8 (0: 2) */
    uint64_t reserved[3];
} qcz_config;

/* Gate record, 88 bytes.  kind:
 *   0 U1    general 2x2 unitary on `target` (Eq. (6)), applied where every
 *           bit of control_mask is 1 (Eq. (7)); m = u00,u01,u10,u11 as (re,im)
 *   1 DIAG1 diagonal phases d0 (target bit 0), d1 (target bit 1), controlled
 *   2 DIAG2 diagonal phases p[2*bit(target2) + bit(target)], controlled
 *   3 X     Pauli-X on `target`, controlled by control_mask (exact)
 *   4 MCZ   sign flip where every bit of control_mask is 1 (exact)
 * The target may not be in control_mask; matrix entries must be finite.   */
typedef struct {
    uint32_t kind;
    uint32_t target;
    uint32_t target2;
    uint32_t reserved;
    uint64_t control_mask;
    double m[8];
} qcz_gate;

typedef struct {
    uint64_t compressed_bytes;   /* sum over chunks of the 4-byte padded stream size: sum sizeof(CB_i) of Eq. (8) */
    uint64_t table_bytes;        /* chunk table, 8 bytes per chunk */
    uint64_t total_bytes;        /* compressed + table; Eq. (8)'s decompressed term is 0 here: decoded chunks live in LDS */
    uint64_t raw_bytes;          /* 2^(n+4) */
    uint64_t arena_bytes;        /* capacity of one arena */
    uint64_t arena_used;         /* arena bytes in use, garbage included */
    uint64_t nchunks;
    uint64_t gates_applied;
    uint64_t lossy_steps;        /* gates that recompressed a chunk at a lossy level */
    uint64_t min_compressed;     /* over the run, after each gate */
    uint64_t max_compressed;
    uint64_t compactions;
    int32_t level;               /* current global level */
    int32_t reserved;
    double ratio;                /* raw_bytes / total_bytes */
    double fidelity_lower_bound; /* prod over lossy gates of (1 - delta), Sec. 3.8 Eq. (11) */
} qcz_footprint_t;

/* Work counters over the committed gates since creation or the last
 * qcz_reset_stats (what the fused kernels moved and, with QCZ_FLAG_TIMING,
 * how long they ran). */
typedef struct {
    uint64_t gate_launches;     /* fused decompress-gate-recompress kernels */
    uint64_t permute_launches;  /* chunk-table permutations (X on chunk-index qubits) */
    uint64_t chunks_reencoded;
    uint64_t amps_touched;      /* chunks_reencoded * amplitudes per chunk */
    uint64_t bytes_read;        /* compressed stream bytes read (4-byte padded) */
    uint64_t bytes_written;     /* compressed stream bytes written (4-byte padded) */
    uint64_t table_bytes;       /* chunk-table and undo-log bytes: 24 per re-encoded chunk */
    uint64_t timed_launches;    /* fused kernels timed with events */
    double gate_kernel_ms;      /* their summed event time */
    uint32_t chunk_waves;       /* launch shape in use: wavefronts per chunk */
    uint32_t grid;              /* launch shape in use: workgroups per fused launch */
    uint32_t tuning;            /* 1 while the autotuner is still measuring */
    uint32_t stops;             /* batches stopped on the device (budget or arena full) and rolled back */
    uint64_t range_gates;       /* gates run in job ranges because their new streams did not fit at once */
    uint64_t cache_gates;       /* QCZ_FLAG_CACHE: gates run through the block cache (event timing, if on,
                                   covers the cache's planning and copy kernels and both job launches) */
    uint64_t cache_hits;        /* chunks whose new stream was copied from an identical job's */
    uint32_t cache_on;          /* 1 while the block cache is in use */
    uint32_t reserved;
    uint64_t range_launches;    /* fused kernels of gates run in job ranges (QCZ_FLAG_TIMING: event-timed and
                                   counted in timed_launches / gate_kernel_ms) */
    uint64_t sweep_gates;       /* gates run as sweeps: their new streams did not fit beside the live ones,
                                   so one launch wrote every chunk into the other arena (the chunks the gate
                                   leaves unchanged copied as they are) and the arenas swapped roles */
    /* the same counters by kind of pass, [0] one gate, [1] a fused run of single-chunk gates (QCZ_FLAG_FUSE),
       [2] a chunk-group run (QCZ_FLAG_GROUPS): event-timed launches and their time (QCZ_FLAG_TIMING), and
       the stream bytes read and written plus table bytes of the committed passes */
    uint64_t kind_launches[3];
    double kind_kernel_ms[3];
    uint64_t kind_bytes[3];
} qcz_stats_t;

/* Bytes of device pool needed for a configuration (state |0..0> plus
 * metadata); larger pools leave room for less compressible states. */
size_t qcz_pool_bytes_min(const qcz_config *cfg);

/* Create the state |0...0> (Sec. 3.3: the state is created in blocks and
 * compressed) inside the caller's device pool.  hip_stream may be NULL (the
 * default stream).  Errors: QCZ_E_INVAL (configuration), QCZ_E_NOMEM (pool
 * smaller than qcz_pool_bytes_min), QCZ_E_DEVICE. */
qcz_status qcz_create(const qcz_config *cfg, void *dev_pool, size_t pool_bytes, void *hip_stream, qcz_state **out);

/* Apply n_gates gate records (host array, copied before return).  The state
 * advances gate by gate; each gate is one timestep of Sec. 3.7.  On
 * QCZ_E_NOMEM (no level fits the budget) or any error, the state is the one
 * after the last gate that completed and *applied (if not NULL) holds their
 * number.  Records are validated first: QCZ_E_INVAL applies nothing. */
qcz_status qcz_apply_gates(qcz_state *st, const qcz_gate *gates, size_t n_gates, size_t *applied);

/* Readout of the state the simulator holds (the amplitudes a_i of Sec. 2.1,
 * Eq. (3), as decompressed from the stored chunks; a full-state simulator
 * gives access to every amplitude at any point of the circuit, Sec. 2.2).  Amplitudes at the k indices idx[]
 * (host, each < 2^n; QCZ_E_INVAL otherwise, nothing written) into
 * out_re_im[2k] (host, re then im per index).  Decompression only: the state
 * is not changed. */
qcz_status qcz_read_amplitudes(qcz_state *st, const uint64_t *idx, size_t k, double *out_re_im);

/* Decode chunks [first_chunk, first_chunk + n_chunks) into device memory
 * dev_out (n_chunks * C doubles, interleaved re/im). */
qcz_status qcz_decode_chunks_to(qcz_state *st, uint64_t first_chunk, uint64_t n_chunks, void *dev_out);

/* Sums over the decoded state: out[0] = sum re, out[1] = sum im,
 * out[2] = sum |a|^2 (fp64 device reductions, fixed order for a given
 * configuration). */
qcz_status qcz_moments(qcz_state *st, double out[3]);

/* Measurement in the computational basis (Sec. 2.1: |a_i|^2 of Eq. (3) is the
 * probability of outcome i, and they sum to 1, Eq. (4)), without collapsing
 * the state.
 * Draw `shots` basis indices (host out_idx) with probability
 * |a_i|^2 / sum |a|^2.  Shot k uses
 * u_k = (SplitMix64 output k for state `seed`) >> 11, times 2^-53, and
 * t = u_k * (sum over chunks of their squared norms, in chunk order): the
 * chunk is the first whose running norm exceeds t, the amplitude the first
 * in it whose running |a|^2 (index order) exceeds the rest of t (the last
 * nonzero one if rounding runs past the end).  QCZ_E_STATE for a zero state. */
qcz_status qcz_sample(qcz_state *st, uint64_t seed, size_t shots, uint64_t *out_idx);

/* Overlap of two compressed states, the quantity of the fidelity definition
 * of Sec. 3.8, Eq. (9): <a|b> = sum_i conj(a_i) b_i over the decoded states
 * (host outputs); a and b have the same qubit count and chunk size
 * (QCZ_E_INVAL otherwise).  Work runs on a's stream after
 * b's stream is drained; a's and b's scratch areas are used. */
qcz_status qcz_overlap(qcz_state *a, qcz_state *b, double *out_re, double *out_im);

qcz_status qcz_footprint(qcz_state *st, qcz_footprint_t *out);

qcz_status qcz_get_stats(qcz_state *st, qcz_stats_t *out);
qcz_status qcz_reset_stats(qcz_state *st);

/* Set the fused kernel's launch shape: chunk_waves in {2, 4, 8} (0 keeps the
 * current one), grid = workgroups per launch (0 keeps it). QCZ_E_INVAL for
 * an unsupported shape. Does not change any result. */
qcz_status qcz_set_launch(qcz_state *st, uint32_t chunk_waves, uint32_t grid);

/* Copy chunk `chunk`'s stream to host memory (capacity cap); *len gets its
 * size.  QCZ_E_INVAL if cap is too small. */
qcz_status qcz_export_chunk(qcz_state *st, uint64_t chunk, void *host_buf, size_t cap, size_t *len);

/* Replace chunk `chunk` by a stream (checkpoint reload).  The header is
 * checked; QCZ_E_FORMAT if it is not a valid stream header or too long. */
qcz_status qcz_import_chunk(qcz_state *st, uint64_t chunk, const void *host_buf, size_t len);

/* Whole-state checkpoint image (Sec. 3.5), one copy each way.  Export:
 * sizes (n_chunks values, host) gets every chunk's stream size and *total the
 * image size, sum over chunks of the size rounded up to 16 bytes; with
 * host_buf null nothing else happens (a size query), otherwise the state is
 * first compacted (its streams packed in chunk order) and the image copied:
 * chunk c's stream starts at the sum of the rounded sizes of chunks < c, and
 * the bytes between a stream's end and its 16-byte boundary are zero.
 * QCZ_E_INVAL if cap < *total.  Import: replace every chunk of `st` by the
 * streams of such an image (len = its total, sizes as exported); the streams'
 * headers are checked first (QCZ_E_FORMAT, state unchanged), QCZ_E_NOMEM if
 * the image exceeds one arena.  The ledger is not part of the image: an import
 * starts a fresh one (no gates applied, bound 1, the configuration's level;
 * QCZ_MODE_PERBLOCK: the squared norm of the imported state) and makes a state
 * left invalid by a failed ranged gate usable again; qcz_resume restores a
 * saved ledger. */
qcz_status qcz_export_state(qcz_state *st, void *host_buf, size_t cap, uint32_t *sizes, size_t *total);
qcz_status qcz_import_state(qcz_state *st, const void *host_buf, size_t len, const uint32_t *sizes);

/* Checkpoint resume (Sec. 3.5): after every chunk of a state saved with
 * qcz_export_state (or qcz_export_chunk) has been imported into a fresh state of the same
 * configuration, restore the run's ledger from the qcz_footprint_t taken when
 * the chunks were saved: level, gates applied, lossy steps, min / max
 * compressed bytes and the fidelity lower bound.  The saved record is only
 * read.  QCZ_E_INVAL if its qubit count / chunk count do not match the state
 * or a field is out of range (level, bound outside (0, 1], min > max);
 * QCZ_E_STATE if the imported streams' compressed bytes differ from the
 * record's (not every chunk imported), or in QCZ_MODE_PERBLOCK (its ledger
 * also tracks the stored squared norm, which the record does not carry). */
qcz_status qcz_resume(qcz_state *st, const qcz_footprint_t *saved);

/* Per-block levels (host array of 2^(n - block_log2) values 0..5) used by
 * QCZ_MODE_PERBLOCK; QCZ_E_STATE in other modes. */
qcz_status qcz_set_block_levels(qcz_state *st, const uint8_t *levels);

/* Stream sizes of all chunks into host memory (n_chunks values). */
qcz_status qcz_chunk_sizes(qcz_state *st, uint32_t *out_sizes);

/* Number of chunks and doubles per chunk of a state. */
uint64_t qcz_num_chunks(const qcz_state *st);
uint32_t qcz_chunk_doubles(const qcz_state *st);

const char *qcz_last_error(const qcz_state *st);
void qcz_destroy(qcz_state *st);

/* ---- per-block level selection ------------------------------------------
 * Sec. 3.7 relaxes one error bound for the whole state when memory runs
 * short; these calls choose one bound per block instead.  The Sec. 3.8
 * argument carries over when each block b is truncated at relative error
 * delta_b per value: one step keeps the fidelity at least
 * 1 - sum_b w_b delta_b, w_b = the block's share of the squared norm.
 * Levels are chosen for a window of gates; gates whose target is a
 * block-index qubit move weight between blocks, but only inside the cosets
 * {b' : b' & ~mix_mask == b & ~mix_mask} of the block-index bits they flip
 * (mix_mask), whose total weight W_c the window conserves.  The per-step
 * budget sum over cosets of W_c * delta(max level in the coset) <= beta
 * therefore holds at every gate of the window and gives at least the
 * Eq. (11) product of a uniform bound beta.  In QCZ_MODE_PERBLOCK the state's ledger
 * (fidelity_lower_bound) multiplies, per gate, 1 - (sum over re-encoded
 * chunks of delta(level) * |chunk before truncation|^2) / |state|^2. */

/* 16 float features per block (device, n_blocks x 16, row major) and the
 * squared norm of each block (device, n_blocks doubles; may be NULL), from
 * the stored values: f0 log2(max(n2_b * n_blocks, 2^-60))/64; f1 zero
 * fraction; f2 (mean biased exponent of nonzero values - 1023)/64; f3
 * exponent range/64; f4..f6 fraction of values whose top 8/16/24 bits equal
 * the previous value's (a chunk's first value is compared with +0.0); f7
 * fraction of sign changes; f8 fraction of chunks stored as two constants;
 * f9 stream bytes / raw bytes of the block; f10 block level/5; f11 (largest
 * biased exponent - 1023)/64 (-17 for an all-zero block); f12
 * max(log10(beta), -20)/5 (-4 for beta = 0); f13 log2(raw / stream bytes of
 * the state)/16; f14 log2(n_blocks)/16; f15 popcount(mix_mask)/16.
 * QCZ_E_INVAL for beta < 0, a mask bit beyond the block index, or blocks of
 * more than 65536 chunks. */
qcz_status qcz_block_stats(qcz_state *st, double beta, uint64_t mix_mask, float *dev_features, double *dev_norms);

/* Padded stream bytes of every block re-encoded at each level: device
 * n_blocks x 6 u64 (block major), overwritten. */
qcz_status qcz_block_level_sizes(qcz_state *st, uint64_t *dev_sizes);

/* Host call, no device work.  Training labels for sizes s[b][l] (host,
 * n_blocks x 6, n_blocks a power of two) and weights w (host, >= 0): each
 * coset c (above; cosets in increasing id b & ~mix_mask, sums in block
 * order) takes the cap level minimising (bytes of its blocks, each at its
 * smallest level <= cap, lowest on ties) + lambda * W_c * delta(cap), lowest
 * cap on ties, for the smallest lambda among 0 and the values where some
 * coset's choice changes whose caps satisfy
 * sum_c W_c delta(cap_c) <= beta * (1 + 2^-20); each block then takes its
 * smallest level under its coset's cap.  Output: levels (host, n_blocks). */
qcz_status qcz_label_levels(const uint64_t *sizes, const double *w, uint64_t n_blocks, double beta,
                            uint64_t mix_mask, uint8_t *levels);

/* Host call.  Budget projection: while sum_c W_c delta(max level in c)
 * exceeds beta * (1 + 2^-20), lower by one every block at the max level of
 * the coset with the largest W_c delta(max level) (lowest id on ties).
 * levels: host, in/out. */
qcz_status qcz_project_levels(const double *w, uint64_t n_blocks, double beta, uint64_t mix_mask,
                              uint8_t *levels);

/* Selector network 16 -> 64 -> 64 -> 6: ReLU hidden layers, softmax over
 * the six levels.  Parameters: 5638 floats on the device, packed W1 (64x16,
 * row major), b1, W2 (64x64), b2, W3 (6x64), b3.  Forward pass over
 * n_samples rows of 16 features (device): probabilities (device,
 * n_samples x 6; may be NULL) and the most probable level (device, u8;
 * may be NULL; lowest level on ties).  Asynchronous on hip_stream. */
qcz_status qcz_mlp_forward(const float *dev_params, const float *dev_x, uint64_t n_samples, float *dev_probs,
                           uint8_t *dev_levels, void *hip_stream);

/* Device workspace bytes that qcz_mlp_train_step needs for n_samples. */
size_t qcz_mlp_workspace_bytes(uint64_t n_samples);

/* One full-batch training step on the device: loss = mean cross-entropy of
 * labels (device u8 in 0..5); dev_grad (5638 floats, may be NULL) receives
 * its gradient; dev_loss (1 float, may be NULL) the loss before the step.
 * step >= 1 then applies Adam step number `step` (beta1 0.9, beta2 0.999,
 * eps 1e-8, bias corrected) to dev_params with moments dev_m / dev_v (5638
 * floats each, zero before step 1); step 0 computes only loss and gradient.
 * dev_work: caller-owned device memory of qcz_mlp_workspace_bytes. */
qcz_status qcz_mlp_train_step(float *dev_params, float *dev_m, float *dev_v, const float *dev_x,
                              const uint8_t *dev_labels, uint64_t n_samples, float lr, uint32_t step,
                              float *dev_grad, float *dev_loss, void *dev_work, size_t work_bytes,
                              void *hip_stream);

/* The training step above without a workspace argument, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * or training loops, harnesses that forbid hipMalloc).  Same arguments,
 * kernels and results as qcz_mlp_train_step; the workspace is a static device
 * array that the library holds on every GPU it runs on until the process
 * ends, sized for QCZ_MLP_NOALLOC_MAX_SAMPLES samples (about 8.5 MiB).  The
 * call allocates nothing.  QCZ_E_NOMEM (nothing launched) for n_samples
 * above that limit, QCZ_E_INVAL as qcz_mlp_train_step.  All calls on one GPU
 * share its array: calls that overlap on one GPU (other streams, other
 * threads) race and must be serialized by the caller. */
#define QCZ_MLP_NOALLOC_MAX_SAMPLES 8192
qcz_status qcz_mlp_train_step_noalloc(float *dev_params, float *dev_m, float *dev_v, const float *dev_x,
                                      const uint8_t *dev_labels, uint64_t n_samples, float lr, uint32_t step,
                                      float *dev_grad, float *dev_loss, void *hip_stream);

/* QCZ_MODE_PERBLOCK: block features -> network -> most probable level per
 * block, raised to at least the rule's level (the loosest level with delta
 * <= beta: one bound for every block already meets the budget) -> budget
 * projection with w_b = n2_b / sum n2 and the window's mix_mask -> block
 * levels of the state.  out_levels (host, n_blocks; may be NULL) receives
 * them. */
qcz_status qcz_select_levels(qcz_state *st, const float *dev_params, double beta, uint64_t mix_mask,
                             uint8_t *out_levels);

/* QCZ_MODE_PERBLOCK: make qcz_apply_gates call qcz_select_levels before the
 * first gate and again every `period` gates, each time with the mixing mask
 * of the next `period` gates (targets of U1 and X gates on block-index
 * qubits).  dev_params must stay valid while attached; NULL detaches. */
qcz_status qcz_set_selector(qcz_state *st, const float *dev_params, double beta, uint32_t period);

/* Block-index bits flipped by the gates (targets of U1 and X gates on
 * block-index qubits): the mix_mask of a window of gates. */
uint64_t qcz_mixing_mask(const qcz_state *st, const qcz_gate *gates, size_t n_gates);

/* Make dst hold the same state as src (streams, chunk table, levels, global
 * level, ledger and counters of the footprint).  src is compacted first (its
 * streams move, its state does not change), then its streams and table are
 * copied device to device on dst's stream.  Same n_qubits, block_log2 and
 * mode; QCZ_E_NOMEM if src's streams exceed dst's arena. */
qcz_status qcz_copy_state(qcz_state *dst, qcz_state *src);

/* ---- codec entry points (no state) -------------------------------------- */

/* Largest stream of a chunk of C doubles (bytes). */
size_t qcz_chunk_cap(uint32_t C);

/* Encode n_chunks chunks of C doubles (device, contiguous) at `level` into
 * device slots of slot_bytes bytes each (slot_bytes >= qcz_chunk_cap(C),
 * multiple of 4); stream sizes go to dev_sizes (device, n_chunks u32).
 * C is a power of two in 128 .. 2048.  codec_flags: QCZ_CODEC_ENTROPY lets
 * a chunk take the entropy-coded body (C = 2048 only); QCZ_CODEC_RESHUFFLE
 * stores values in Solution D's order (Sec. 4.2); other bits: QCZ_E_INVAL. */
#define QCZ_CODEC_ENTROPY 1u
#define QCZ_CODEC_RESHUFFLE 2u
/* Solution B (Sec. 4.2), alone (no other codec bit), lossy levels 1..5, C >= 256: each value quantized
 * in the log domain (the bit pattern of |x| read as an integer; bin width 2^(52-t), t = 16, 13, 9, 6, 3
 * for 1e-5 .. 1e-1), predicted from the previous nonzero value of its part (real parts, then imaginary
 * parts), 16,384 symbols (escape, zero, codes -8190 .. 8191) Huffman coded with the sign bit beside each
 * code; header mode 3.  Slots hold qcz_chunk_cap_codec(C, QCZ_CODEC_PREDICT) bytes; a chunk whose
 * stream would not fit its slot gets size 0. */
#define QCZ_CODEC_PREDICT 4u
/* Bytes a slot needs for the streams of a codec (0 for a bad C or flags). */
size_t qcz_chunk_cap_codec(uint32_t C, uint32_t codec_flags);
qcz_status qcz_encode_chunks(const void *dev_in, uint32_t C, uint64_t n_chunks, int level, uint32_t codec_flags,
                             void *dev_slots, size_t slot_bytes, uint32_t *dev_sizes, void *hip_stream);

/* Decode n_chunks streams from device slots into C doubles each (device);
 * streams with and without the entropy stage, in either value order, and
 * Solution B streams (C >= 256).  Streams must be well formed (as the
 * encoders write them): a malformed Solution B stream decodes to unspecified
 * values, without access outside its slot. */
qcz_status qcz_decode_chunks(const void *dev_slots, size_t slot_bytes, const uint32_t *dev_sizes, uint32_t C,
                             uint64_t n_chunks, void *dev_out, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* QCZ_H */

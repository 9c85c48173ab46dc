/*
 * psf.h -- C ABI of the progressive spatio-temporal filtering (PSTF) hash
 * library for AMD Instinct MI355X (gfx950).
 *
 * Method: J. Pantaleoni, "Online path sampling control with progressive
 * spatio-temporal filtering", arXiv 2005.07547.  Each frame (iteration) the
 * caller
 *   1. inserts path-vertex samples into a spatio-directional hash table
 *      (Sec. 2.6): every cell accumulates a sample count and a sum of sample
 *      values, the counter c_h^new and the numerator of Eq. 6 with box basis
 *      functions and MIS weight 1 (Algorithm 1: increment_counters,
 *      update_approx), or, in a weighted table, each record's MIS weight;
 *   2. applies the temporal blend of Sec. 2.4 (Eq. 10-11) to every cell that
 *      received samples: L <- (1 - alpha) L + alpha * mean, with
 *      alpha = max(sqrt(c_new / (c_old + c_new)), 1 / T_max) and the
 *      cumulative count c_old += c_new;
 *   3. queries the filtered approximant at arbitrary vertices (the lookup of
 *      L~^old inside Algorithm 1 and the control-variate term of Eq. 25).
 *
 * Conventions shared by every entry point
 *   - Pointers named d_* (and the arrays inside psf_records / psf_queries)
 *     are DEVICE pointers; everything else is host memory.
 *   - stream is a hipStream_t (0 = the null stream).  Work is enqueued on it
 *     asynchronously unless a function says it synchronises.  A table is
 *     used from one stream at a time; the caller orders its calls.
 *   - Every call returns a psf_status.  Argument errors return before any
 *     work is enqueued; psf_last_error() then describes the problem (a
 *     thread-local string owned by the library).  Kernel launch failures
 *     return PSF_HIP_ERROR; asynchronous device faults surface at the
 *     caller's next synchronisation.
 *   - Data conditions are not errors: non-finite inputs are counted as
 *     skipped, samples for which no slot was found within max_probe probes
 *     (table full) as dropped, and grid coordinates outside the signed
 *     16-bit range as coord_overflow (their key wraps).  See psf_get_stats.
 *   - n = 0 is a no-op that returns PSF_OK.
 */
#ifndef PSF_H_
#define PSF_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* psf_stream;  /* a hipStream_t */

typedef enum psf_status {
  PSF_OK = 0,
  PSF_INVALID_ARGUMENT = 1,
  PSF_OUT_OF_MEMORY = 2,
  PSF_BUFFER_TOO_SMALL = 3,
  PSF_HIP_ERROR = 4,
  PSF_NOT_SUPPORTED = 5
} psf_status;

/* Temporal blend modes (Sec. 2.4).  PAPER is Eq. 11.  CONST is the
 * constant-alpha "exponential weighting" limit and LINEAR the "linear
 * accumulation" limit (no square root) that the same section names.  In
 * every mode a cell blended for the first time (c_old = 0) takes its mean. */
enum { PSF_ALPHA_PAPER = 0, PSF_ALPHA_CONST = 1, PSF_ALPHA_LINEAR = 2 };

/* Storage of the approximant.  The blend always runs in FP32 and the
 * accumulators are FP32; F16 and BF16 round to nearest even on store (F16
 * saturates at +-65504 and counts each saturation).  F16 and BF16 blend from
 * the stored 16-bit value, so every frame re-rounds the state (the error
 * grows to about u * T_max relative, u the format's unit roundoff).  F16_EF
 * and BF16_EF store the same 16-bit approximant, which is what lookups,
 * exports and estimators read, and also carry each channel's FP32 rounding
 * residual in the slot (error feedback): the blend continues from the
 * unrounded FP32 value, so a lookup sees one rounding (relative error
 * <= u in the format's normal range).  The slot is 32 bytes in every
 * format. */
enum {
  PSF_STATE_F32 = 0,
  PSF_STATE_F16 = 1,
  PSF_STATE_BF16 = 2,
  PSF_STATE_F16_EF = 3,
  PSF_STATE_BF16_EF = 4
};

/* psf_reset what-bits.  COUNTERS zeroes every cell's c_old (the global
 * counter reset of Sec. 2.4): cells keep their key but are not reported by
 * queries until blended again, and their next blend starts over with
 * alpha = 1.  CLEAR empties the table.  STATS zeroes the statistics. */
enum { PSF_RESET_COUNTERS = 1u, PSF_RESET_CLEAR = 2u, PSF_RESET_STATS = 4u };

/* Insert strategies (psf_config.insert_mode). */
enum {
  PSF_INSERT_AUTO = 0,        /* library choice: partitioned when the table
                                 has at most 16384 partitions, else direct */
  PSF_INSERT_DIRECT = 1,      /* wave-merged global CAS/atomics per record */
  PSF_INSERT_PARTITIONED = 2  /* bin by table partition, aggregate in LDS */
};

/* psf_config.flags */
enum {
  PSF_FLAG_PROBE_STATS = 1u,   /* record a probe-length histogram */
  PSF_FLAG_TIMING = 2u,        /* bracket every kernel launch with HIP events */
  PSF_FLAG_TRANSPOSE_RUNS = 4u, /* partitioned insert: always transpose the
                                  per-tile run table before the merge pass
                                  (by default only tables of 2^22 entries
                                  or more are transposed) */
  PSF_FLAG_TRACK_VARIANCE = 8u, /* keep a binary32 luminance variance per
                                  cell (below); RGB payload, unweighted
                                  tables only (NOT_SUPPORTED otherwise) */
  PSF_FLAG_NO_ACCUMULATORS = 16u /* a table for the fused calls only (below) */
};

/* Tables without frame accumulators (PSF_FLAG_NO_ACCUMULATORS).  Sec. 2.4's
 * insert and blend of one frame only need a frame's sums between a separate
 * psf_insert_samples and psf_temporal_update; psf_iterate (and
 * psf_progressive_step, psf_iterate_batch) on the partitioned strategy sums
 * a frame in the merge pass's LDS and blends it there.  Such a table leaves
 * out the 16-byte per-slot accumulator (and, with
 * PSF_FLAG_TRACK_VARIANCE, the 8-byte pending squared-luminance sum):
 * 40 bytes per slot for the cell state and key mirror instead of 56.
 * Requirements: RGB payload and an insert_mode other than DIRECT
 * (psf_table_bytes returns 0 and psf_create_table INVALID_ARGUMENT
 * otherwise), and a table narrow enough for the partitioned strategy, at
 * most 2^14 partitions (psf_table_bytes returns 0 and psf_create_table
 * NOT_SUPPORTED otherwise).  On such a table
 * psf_insert_samples and psf_temporal_update return NOT_SUPPORTED, as does
 * psf_iterate with more records than max_batch (a launch that would be
 * split); psf_iterate with no records blends nothing and only answers the
 * queries.  Lookups, resets and exports work as on any table; exported
 * n_new is 0 (no frame is ever pending). */

/* Per-cell luminance variance (PSF_FLAG_TRACK_VARIANCE).  The paper keeps
 * none; this library's reading: the spread of a cell's samples around its
 * approximant under the temporal weights of Eq. 10-11.  With the luminance
 * Y = (r + 2 g + b) / 4 (Y of YCoCg), each blend of a frame with n samples,
 * luminance mean m and population variance s2 (both from binary64 sums of
 * Y and Y^2, rounded once) updates, in binary32, with the frame's alpha and
 * mu the luminance of the state the blend continues from:
 *     V <- (1 - alpha) V + alpha (s2 + (1 - alpha) (m - mu)^2)
 * (alpha = 1, a cell's first blend or one after a counter reset: V = s2).
 * V is then the population variance of every sample the cell has blended,
 * frame j's samples each weighted beta_j / n_j (beta_j the weight Eq. 10-11
 * gives frame j's mean in the approximant).  Memory: 12 more bytes per slot
 * and 4 per staged entry.  The partitioned insert stages each entry's sum
 * of squared luminances (records of one cell in neighbouring pixels are
 * pre-merged as in other tables with the default 8 records per binning
 * thread; with more, each record stays an entry of its own) and its merge
 * pass holds a further binary64 sum per slot in LDS (46 instead of 38
 * bytes). */

/* Kernel kinds reported by psf_kernel_times. */
enum {
  PSF_K_KEYS = 0,
  PSF_K_INSERT_DIRECT = 1,
  PSF_K_BIN = 2,
  PSF_K_MERGE = 3,
  PSF_K_MERGE_BLEND = 4,
  PSF_K_UPDATE = 5,
  PSF_K_QUERY = 6,
  PSF_K_BATCH = 7,
  PSF_K_TRANSPOSE = 8,
  PSF_K_ESTIMATE = 9,
  PSF_K_STEP = 10,
  PSF_K_COUNT = 11
};

/*
 * Table configuration.  The cell key (spatio-directional hashing, Sec. 2.6;
 * this library's fixed specification, identical on every implementation):
 *   level  l = clamp(floor(e / 2), 0, max_level), e the binary32 exponent of
 *             kappa * |p - cam|^2 (no square root or logarithm; kappa = 0
 *             selects l = 0).  With kappa = (k_s * theta_pixel / 2^e_min)^2
 *             the cell edge 2^(e_min + l) tracks k_s pixel footprints at the
 *             vertex's camera distance (the level hierarchy of Sec. 2.3).
 *   coords (ix, iy, iz) = floor(p * 2^-(e_min + l)), kept modulo 2^16.
 *   normal octahedral bin on a 2^normal_bins_log2 square grid.
 *   glossy vertices (roughness array given and roughness < rough_thr, strict)
 *             also key the outgoing direction on a 2^dir_bins_log2 grid.
 *   key = l<<59 | glossy<<58 | dir_bin<<52 | normal_bin<<48 | iz<<32 | iy<<16 | ix
 * Bit 63 of a key is always 0; the key is injective on cells while no
 * coordinate overflows, so the stored key is its own checksum.
 */
typedef struct psf_config {
  uint32_t log2_slots;       /* 4..30: table of 2^log2_slots slots */
  uint32_t max_probe;        /* 1..2^log2_slots: linear-probe bound */
  float cam[3];              /* camera position for the level rule */
  float kappa;               /* >= 0, finite; 0 = fixed level 0 */
  int32_t e_min;             /* finest cell edge 2^e_min, -100..100 */
  int32_t max_level;         /* 0..15 */
  int32_t normal_bins_log2;  /* 0..2 */
  int32_t dir_bins_log2;     /* 0..3 */
  float rough_thr;           /* glossy iff roughness < rough_thr */
  int32_t alpha_mode;        /* PSF_ALPHA_* */
  float alpha;               /* CONST mode alpha, (0, 1] */
  float t_max;               /* PAPER mode temporal window, >= 1 */
  int32_t state_dtype;       /* PSF_STATE_* */
  uint32_t flags;            /* PSF_FLAG_* */
  int32_t insert_mode;       /* PSF_INSERT_* */
  uint32_t part_log2;        /* partitioned insert: log2 slots per partition
                                (0 = default: 11, or 12 for tables of 2^25
                                slots or more; else 8..12.  With
                                PSF_FLAG_TRACK_VARIANCE or weighted = 1:
                                default 10, or 11 for tables of 2^24
                                slots or more; at most 11).  A table of
                                more than 16384 partitions takes the direct
                                strategy. */
  uint64_t max_batch;        /* partitioned insert: records binned per launch
                                (0 = default 4M, at most 2^31); larger
                                inserts are split */
  uint32_t bin_per;          /* partitioned insert: records per thread of the
                                binning pass (0 = default 8, else 8, 12, 16);
                                a binning tile is 512 * bin_per records */
  uint32_t weighted;         /* 0: every record counts 1 (integer counters).
                                1: MIS-weighted counters (Eq. 5-6 with
                                weights w != 1, e.g. a down-weighted field
                                that keeps only some sampling techniques,
                                Sec. 2.5): records may carry a weight array;
                                a cell's counter is the binary32 sum of the
                                weights that fell on it and its sample mean
                                the weighted mean; Eq. 11 takes the weighted
                                counters.  The partitioned insert sums a
                                frame's weights in binary64 and rounds the
                                sum once (the same bits on every run); the
                                direct insert adds them with binary32
                                atomics (like its value sums, the result
                                depends on their order). */
  uint32_t payload;          /* PSF_PAYLOAD_RGB: the approximant is an RGB
                                triple per cell.  PSF_PAYLOAD_SH2_YCOCG:
                                luminance as two spherical-harmonic bands
                                over the normal plus YCoCg chroma (below);
                                F32 state and the direct insert strategy
                                only (NOT_SUPPORTED otherwise). */
} psf_config;

/* Cell payloads.  SH2_YCOCG (Sec. 2.6: normal variation within a cell as
 * two SH bands of luminance in a YCoCg colour decomposition), this
 * library's reading of the unspecified projection: each frame fits, per
 * cell, the four band-0/1 luminance coefficients (real SH, basis
 * 1/(2 sqrt(pi)) and sqrt(3/(4 pi)) (n_y, n_z, n_x)) to the samples by
 * weighted least squares over their normals, in binary64, with a ridge of
 * 1e-7 times the cell's weight on the band-1 coefficients (the system is
 * always definite; a constant field is reproduced exactly; a cell whose
 * normals are all equal reproduces its mean at that normal), and takes the
 * weighted mean of the chroma pair (Co, Cg); these six numbers are the
 * cell's state (24 bytes), blended by Eq. 10-11 with the cell's counters.
 * A lookup evaluates the luminance at the query's normal and returns RGB
 * (R = Y + Co - Cg, G = Y + Cg, B = Y - Co - Cg).  Key the cells with
 * normal_bins_log2 = 0 to let the payload, not the key, carry the normal. */
enum { PSF_PAYLOAD_RGB = 0, PSF_PAYLOAD_SH2_YCOCG = 1 };

/* Vertex records, structure of arrays, N float32 each (device memory).
 * ox..oz is the outgoing direction omega_o (pointing back along the path,
 * Algorithm 1); it is read only for glossy vertices.  rough may be NULL
 * (every vertex diffuse).  r, g, b is the sample value assembled by the
 * caller (the path tail estimate of Eq. 3 / Eq. 9).  footprint may be NULL;
 * otherwise it is the width of the path's footprint at each vertex (Sec.
 * 2.3 selects the hierarchy level by footprint) and the level is the
 * largest l <= max_level with 2^(e_min + l) <= footprint (0 below 2^e_min)
 * instead of the camera-distance rule; a non-finite or non-positive
 * footprint rejects the record like a non-finite position.  weight may be
 * NULL (every weight 1); otherwise it is the record's MIS weight (Eq. 5:
 * the record adds w to its cell's counter and w * (r, g, b) to its sum) and
 * the table must have been created with weighted = 1 (INVALID_ARGUMENT
 * otherwise).  A weight that is not finite and > 0 rejects the sample (it
 * is counted as skipped; as a query vertex of psf_iterate the record is
 * still answered). */
typedef struct psf_records {
  const float *px, *py, *pz;
  const float *nx, *ny, *nz;
  const float *ox, *oy, *oz;
  const float *r, *g, *b;
  const float *rough;
  const float *footprint;
  const float *weight;
} psf_records;

/* Query vertices: the same fields without a sample value. */
typedef struct psf_queries {
  const float *px, *py, *pz;
  const float *nx, *ny, *nz;
  const float *ox, *oy, *oz;
  const float *rough;
  const float *footprint;
} psf_queries;

typedef struct psf_stats {
  uint64_t submitted;       /* records passed to insert calls */
  uint64_t skipped;         /* non-finite records (inserts and queries are
                               counted separately: this is inserts) */
  uint64_t dropped;         /* records with no slot within max_probe */
  uint64_t coord_overflow;  /* inserted records with a wrapped coordinate */
  uint64_t touched_last;    /* cells blended by the last temporal update */
  uint64_t touched_total;   /* cells blended, summed over updates */
  uint64_t updates;         /* temporal updates applied */
  uint64_t saturated;       /* F16 stores clamped to +-65504 */
  uint64_t occupied;        /* non-empty slots (computed on request) */
  uint64_t probe_hist[16];  /* with PSF_FLAG_PROBE_STATS: probes needed per
                               cell insertion, bucket min(probes-1, 15) */
} psf_stats;

typedef struct psf_table psf_table;

/* Bytes of device memory a table with this configuration needs (slots,
 * accumulators, touched list, staging, statistics).  0 if cfg is invalid. */
size_t psf_table_bytes(const psf_config* cfg);

/* Create a table.  device_buffer (nullable) is caller-owned device memory of
 * at least psf_table_bytes(cfg) bytes, 256-byte aligned, that must outlive
 * the table; when NULL the library allocates.  The table is initialised
 * (all slots empty) on stream.  BUFFER_TOO_SMALL if buffer_bytes is short. */
psf_status psf_create_table(const psf_config* cfg, void* device_buffer, size_t buffer_bytes,
                            psf_stream stream, psf_table** out);

/* Frees what the library allocated.  When the library allocated the
 * table's device memory it first synchronises the table's last stream.  A
 * caller-owned device_buffer is not waited for: work already enqueued on the
 * table's stream still uses it, so the caller reuses or frees it only in
 * that stream's order (or after synchronising), as with any stream-ordered
 * allocation.  NULL is a no-op. */
psf_status psf_destroy(psf_table* t);

/* Scatter n records into the table (Eq. 5-6 accumulation; Algorithm 1's
 * increment_counters / update_approx).  May be called several times before
 * a temporal update; contributions add up. */
psf_status psf_insert_samples(psf_table* t, const psf_records* rec, uint64_t n, psf_stream stream);

/* Fold every touched cell's mean into its approximant (Eq. 10-11), add its
 * count to c_old and clear its accumulator.  Untouched cells are unchanged. */
psf_status psf_temporal_update(psf_table* t, psf_stream stream);

/* Look up n query vertices.  d_out_rgb receives 3*n floats, SoA (all r, then
 * all g, then all b); d_out_found (nullable) receives n bytes, 1 where the
 * query's cell exists and has been blended (c_old > 0), else 0 with a zero
 * output.  Reads the state left by the last completed temporal update. */
psf_status psf_query(psf_table* t, const psf_queries* q, uint64_t n, float* d_out_rgb,
                     uint8_t* d_out_found, psf_stream stream);

/* Multi-level lookup (Sec. 2.3: the finite elements form a hierarchy of
 * levels).  As psf_query, but a query vertex whose own cell has no blended
 * value is answered by the finest coarser cell that has one (the same
 * normal and direction bins at levels l + 1 .. l + levels_up, up to
 * max_level).  d_out_level (nullable, n bytes) receives 0 where no level
 * answered, else 1 + the number of levels above the vertex's own.
 * levels_up <= 15; 0 is psf_query. */
psf_status psf_query_levels(psf_table* t, const psf_queries* q, uint64_t n, uint32_t levels_up,
                            float* d_out_rgb, uint8_t* d_out_level, psf_stream stream);

/* One whole iteration: insert rec, temporal update, then query q.  Same
 * result as the three calls in sequence; when the table has no pending
 * inserts the partitioned strategy fuses insert and blend in one pass, and
 * when q is rec itself (the same arrays, nq == n) that pass also hands every
 * record its cell's new value, so the query costs no second lookup. */
psf_status psf_iterate(psf_table* t, const psf_records* rec, uint64_t n, const psf_queries* q,
                       uint64_t nq, float* d_out_rgb, uint8_t* d_out_found, psf_stream stream);

/* One step of the progressive solver (Sec. 2.2, Eq. 8-9; Algorithm 1): at
 * each of n path vertices x_i the new sample is
 *
 *   Lbar_i = L_e(x_i) + L~(x_{i+1}) * t_i
 *
 * where L~(x_{i+1}) is the approximant at the path's next vertex as
 * psf_query returns it (the state of the last completed update: the
 * previous frame's approximant; 0 where the next vertex has no blended cell
 * or no valid key, e.g. a path that ended) and t_i = f G w / p is the
 * caller's throughput factor of the sampled step x_i -> x_{i+1}.  The
 * samples are written to d_samples (3*n floats, SoA, caller-owned device
 * memory), inserted at the vertices x and blended, as psf_iterate with no
 * queries would.  x->r, g, b are ignored; le may be NULL (no emission).
 * Algorithm 2's field L_o\e (radiance minus emission) is the same step with
 * the emission the sampled step picks up at x_{i+1} (times t_i, plus any
 * next-event estimate at x_i) passed as le. */
typedef struct psf_step_args {
  const float *le_r, *le_g, *le_b;  /* emission at x_i (all three or none) */
  const float *t_r, *t_g, *t_b;     /* throughput factor f G w / p */
} psf_step_args;

psf_status psf_progressive_step(psf_table* t, const psf_records* x, const psf_queries* next,
                                const psf_step_args* a, uint64_t n, float* d_samples,
                                psf_stream stream);

/* Reset (PSF_RESET_* bits). */
psf_status psf_reset(psf_table* t, uint32_t what, psf_stream stream);

/* Local counter reset (Sec. 2.4: besides globally, counters may be zeroed
 * locally and on demand, where the caller's heuristic detects a change).
 * Every cell whose box [i*s, (i+1)*s) per axis (s = 2^(e_min + level), i the
 * cell's grid coordinates as stored, signed 16-bit) meets the closed box
 * [lo, hi] gets c_old = 0, as PSF_RESET_COUNTERS does for every cell: it is
 * not reported by queries until blended again, and that blend starts over
 * with alpha = 1.  Pending samples stay.  lo and hi are host arrays of three
 * finite floats with lo <= hi; the test is done in binary32 (exact here:
 * the box corners are integers times powers of two). */
psf_status psf_reset_region(psf_table* t, const float* lo, const float* hi, psf_stream stream);

/* Keys of n records (all ones for rejected records); test support. */
psf_status psf_compute_keys(psf_table* t, const psf_records* rec, uint64_t n, uint64_t* d_out_keys,
                            psf_stream stream);

/* Statistics into *out (host).  Synchronises stream. */
psf_status psf_get_stats(psf_table* t, psf_stats* out, psf_stream stream);

/* Copy every occupied cell to host arrays of capacity cap: keys, pending
 * counts n_new, cumulative counts c_old (for a weighted table both hold
 * binary32 bit patterns: weight sums), approximant (3*cap floats, SoA,
 * decoded to float).  Any output pointer except keys may be NULL.  *count
 * receives the number of occupied cells; BUFFER_TOO_SMALL if it exceeds cap
 * (nothing is written then).  Order is unspecified.  Synchronises stream. */
psf_status psf_export_cells(psf_table* t, uint64_t* keys, uint32_t* n_new, uint32_t* c_old,
                            float* state_rgb, uint64_t cap, uint64_t* count, psf_stream stream);

/* Allocation-free variant of psf_export_cells, for callers that cannot
 * allocate device memory (tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments, results and errors, but the device
 * staging of the compacted cells lives in a fixed array the library holds
 * on each GPU for the life of the process (28 MiB + 256 B) instead of a
 * per-call allocation.  At most 1048576 occupied cells: a table with more
 * returns PSF_NOT_SUPPORTED (after setting *count), before anything is
 * compacted.  Every call on one GPU shares that GPU's array, so calls that
 * overlap on one GPU (from several threads or streams) race; the caller
 * serialises them.  Synchronises stream. */
psf_status psf_export_cells_noalloc(psf_table* t, uint64_t* keys, uint32_t* n_new, uint32_t* c_old,
                                    float* state_rgb, uint64_t cap, uint64_t* count, psf_stream stream);

/* Luminance variance of every occupied cell (a table created with
 * PSF_FLAG_TRACK_VARIANCE, else NOT_SUPPORTED): keys and variance into host
 * arrays of capacity cap.  Pending frame sums are not included.  Otherwise
 * as psf_export_cells.  Synchronises stream. */
psf_status psf_export_variance(psf_table* t, uint64_t* keys, float* var, uint64_t cap, uint64_t* count,
                               psf_stream stream);

/* Export of an SH2_YCOCG table: keys, c_old and the six state numbers per
 * occupied cell into host arrays of capacity cap (coeff: 6 * cap floats,
 * SoA: the four luminance coefficients, then Co, then Cg).  Pending frame
 * sums are not exported.  Otherwise as psf_export_cells (NOT_SUPPORTED for
 * an RGB table).  Synchronises stream. */
psf_status psf_export_sh_cells(psf_table* t, uint64_t* keys, uint32_t* c_old, float* coeff, uint64_t cap,
                               uint64_t* count, psf_stream stream);

/* Batched form: one iteration (insert, temporal update, query) of k
 * independent sessions, each with its own table, in three launches that
 * cover every session (binning, merge + blend, lookup).  Each session's
 * result equals the same session run alone through psf_iterate.  Sessions
 * that cannot join the batch (direct insert strategy, samples pending from
 * psf_insert_samples, n above the table's max_batch, a binning width
 * different from the first batchable session's, partitions wider than both
 * 2^11 slots and the narrowest batchable session's) run through psf_iterate
 * first, on the same stream.  d_out_rgb (3*nq floats, SoA) and d_out_found
 * (nullable) as in psf_query; queries equal to the records (the same
 * arrays) are answered by the merge pass, as in psf_iterate. */
typedef struct psf_session {
  psf_table* table;
  psf_records rec;
  uint64_t n;
  psf_queries q;
  uint64_t nq;
  float* d_out_rgb;
  uint8_t* d_out_found;
} psf_session;

/* A batch context owns the session descriptors of batched calls: a pinned
 * host copy and a device copy of up to max_sessions entries.  A call made
 * during HIP stream capture records a copy from the pinned buffer, so a
 * context used in a captured graph must not be used for other calls while
 * the graph is replayed (use one context per graph).  Outside capture, a
 * call waits for the context's previous descriptor copy before reusing the
 * pinned buffer.  Host-side statistics (submitted, updates) count calls,
 * not graph replays. */
typedef struct psf_batch psf_batch;

psf_status psf_batch_create(uint32_t max_sessions, psf_batch** out);

/* Synchronises the context's last descriptor copy and frees it; NULL is a
 * no-op. */
psf_status psf_batch_destroy(psf_batch* b);

psf_status psf_iterate_batch(psf_batch* b, const psf_session* sessions, uint32_t k, psf_stream stream);

/* Estimators built on two fields (Sec. 2.5): t_oe holds the approximant of
 * L_o\e (outgoing radiance minus emission, the field Algorithm 2 tracks),
 * keyed on the outgoing direction; t_fli holds the approximant of f L_i
 * (incoming radiance times the BSDF), keyed on the incoming (sampled)
 * direction.  For the latter the key should carry the direction at every
 * vertex: create t_fli with rough_thr = +INFINITY and pass roughness.
 *
 * At each of n path vertices (SoA device arrays, caller-owned) the call
 * looks up L~o\e(x, w_o) in t_oe and f~L_i(x, w_i) in t_fli, as psf_query
 * would, and combines them with the vertex's Monte Carlo sample
 * g = L_i(x, w_i) f(w_i, w_o) (gr, gg, gb) and its weight wp = w / p_perp
 * (MIS weight over the projected-solid-angle density of w_i):
 *
 *   PSF_EST_CV      (Sec. 4.2, Eq. 25; param = beta):
 *                   wp * (g - beta f~L_i) + beta L~o\e
 *   PSF_EST_BIASED  (Sec. 5, Eq. 28; param = gamma):
 *                   gamma * wp * (g - f~L_i) + L~o\e
 *
 * The known integral L~o\e of the control variate is added once, outside
 * the wp factor (the unbiased form; the printed estimators put it inside).
 * Where either cell is missing (or not yet blended) the vertex gets the
 * plain estimate wp * g and d_out_applied (nullable, n bytes) is 0; else 1.
 * d_out_rgb receives 3*n floats, SoA.  Arithmetic is binary32 in the order
 * written, without contraction.  Reads the state left by each table's last
 * completed temporal update.  param must be finite. */
enum {
  PSF_EST_CV = 0,
  PSF_EST_BIASED = 1
};

typedef struct psf_estimate_args {
  const float *px, *py, *pz;     /* vertex position */
  const float *nx, *ny, *nz;     /* shading normal */
  const float *oox, *ooy, *ooz;  /* outgoing direction w_o (key of t_oe) */
  const float *oix, *oiy, *oiz;  /* incoming, sampled direction w_i (key of t_fli) */
  const float *rough;            /* nullable: all vertices diffuse */
  const float *gr, *gg, *gb;     /* sample g = L_i f */
  const float *wp;               /* w / p_perp */
  const float *footprint;        /* nullable: levels as in psf_records */
} psf_estimate_args;

psf_status psf_estimate(psf_table* t_oe, psf_table* t_fli, const psf_estimate_args* a, uint64_t n,
                        int32_t mode, float param, float* d_out_rgb, uint8_t* d_out_applied,
                        psf_stream stream);

/* Path sampler for the progressive solver (Sec. 2.2, Eq. 7-9; Algorithms 1
 * and 2): the step upstream of the hash path, on the GPU.  Traces one path
 * of `verts` vertices x_1..x_V per pixel sample through a scene of quads
 * and spheres with Lambertian materials and writes, per vertex (depth-major:
 * vertex 1 of every path, then vertex 2, ...; n = paths * verts entries per
 * array, caller-owned device memory), what one solver frame consumes:
 *   x        the vertex as a record: position, normal (facing the outgoing
 *            direction), outgoing direction omega_o = -omega_i of the step
 *            that reached it, roughness (of its primitive);
 *   next     its next vertex x_{i+1} as a query (NaN position where the
 *            path left the scene: its lookup finds nothing);
 *   t        the throughput factor f G w / p of the sampled step x_i ->
 *            x_{i+1} (cosine-weighted scattering: the albedo; 0 after an
 *            escape);
 *   le       the emission argument of psf_progressive_step:
 *              PSF_PATHS_LO  (Algorithm 1, field L_o):   L_e(x_i);
 *              PSF_PATHS_LOE (Algorithm 2, field L_o\e): w_nee NEE(x_i) +
 *                t_i w_bsdf L_e(x_{i+1}), next-event estimation toward a
 *                uniformly chosen emitter (uniform point on it, shadow ray)
 *                and the emission reached by the scattering event, combined
 *                by the balance heuristic.
 * So psf_sample_paths followed by psf_progressive_step(x, next, {le, t}) is
 * one frame of the solver, entirely on the device.  A path that leaves the
 * scene restarts from its origin (every path has exactly verts vertices).
 * Random numbers: Philox-4x32-10 keyed (seed, frame) with counter (path,
 * vertex, purpose, 0), so the output is a pure function of its inputs.
 * Emitters emit on both sides of quads and outward from spheres, with
 * radiance `emission` (uniform, Lambertian). */
enum { PSF_PRIM_QUAD = 0, PSF_PRIM_SPHERE = 1 };
enum { PSF_PATHS_LO = 0, PSF_PATHS_LOE = 1 };
enum { PSF_ORIGIN_CAMERA = 0, PSF_ORIGIN_POINT = 1 };

typedef struct psf_prim {
  int32_t kind;        /* PSF_PRIM_* */
  float p[3];          /* quad: centre; sphere: centre */
  float u[3];          /* quad: half-edge vector (the quad is p + a u + b v,
                          |a|, |b| <= 1); sphere: u[0] = radius */
  float v[3];          /* quad: the other half-edge vector */
  float albedo[3];     /* Lambertian reflectance, f = albedo / pi */
  float emission[3];   /* emitted radiance (0 for no emitter) */
  float rough;         /* reported as the vertex roughness (keys glossy
                          vertices by direction); scattering is diffuse */
} psf_prim;

typedef struct psf_camera {
  float pos[3];        /* origin of every path */
  float fwd[3], up[3]; /* unit, orthogonal: view direction and image up */
  float fov_y;         /* vertical field of view, radians, in (0, pi) */
  uint32_t width, height, spp;  /* paths = width * height * spp, pixel =
                                   path / spp in scanline order */
} psf_camera;

typedef struct psf_path_params {
  uint32_t verts;      /* vertices per path, >= 1 */
  int32_t mode;        /* PSF_PATHS_LO or PSF_PATHS_LOE */
  int32_t origin;      /* PSF_ORIGIN_CAMERA: pinhole camera rays, jittered
                          in the pixel; PSF_ORIGIN_POINT: uniform directions
                          from cam.pos (a closed scene seen from inside) */
  uint32_t seed, frame;
} psf_path_params;

typedef struct psf_path_out {
  float *px, *py, *pz, *nx, *ny, *nz, *ox, *oy, *oz, *rough;          /* x_i */
  float *qx, *qy, *qz, *qnx, *qny, *qnz, *qox, *qoy, *qoz, *qrough;   /* x_{i+1} */
  float *t_r, *t_g, *t_b;                                             /* f G w / p */
  float *le_r, *le_g, *le_b;                                          /* emission argument */
} psf_path_out;

/* d_prims: n_prims scene primitives in device memory (at most 4096; a
 * kind other than PSF_PRIM_SPHERE is read as a quad).  INVALID_ARGUMENT for
 * a NULL output array, verts = 0, an unknown mode or origin, a field of
 * view outside (0, pi), an empty image or more than 2^32 paths. */
psf_status psf_sample_paths(const psf_prim* d_prims, uint32_t n_prims, const psf_camera* cam,
                            const psf_path_params* p, const psf_path_out* out, psf_stream stream);

/* Philox-4x32-10 (Salmon et al., SC'11) on the device, as the path sampler
 * uses it: out[4i..4i+3] = philox(ctr[4i..4i+3], key[2i..2i+1]) for i < n
 * (device arrays); test support for the generator's known answers. */
psf_status psf_philox(const uint32_t* d_ctr, const uint32_t* d_key, uint64_t n, uint32_t* d_out, psf_stream stream);

/* Per-kernel timing (tables created with PSF_FLAG_TIMING): for each kernel
 * kind k < PSF_K_COUNT, launches[k] and total_ms[k] (host arrays of
 * PSF_K_COUNT entries) receive the launches recorded since the last reset
 * and their summed HIP-event durations, measured on the stream each kernel
 * ran on.  reset != 0 clears the record.  Synchronises the recorded events.
 * At most 8192 launches are kept; older ones are folded into the sums as
 * the ring wraps.  NOT_SUPPORTED without PSF_FLAG_TIMING. */
psf_status psf_kernel_times(psf_table* t, uint64_t* launches, double* total_ms, int reset);

/* Name of kernel kind k ("" if out of range). */
const char* psf_kernel_name(uint32_t k);

/* Description of the last error on this thread ("" if none). */
const char* psf_last_error(void);

/* Library version string. */
const char* psf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PSF_H_ */

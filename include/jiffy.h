/*
 * jiffy.h -- C ABI of the MI355X (gfx950) Jiffy LiDAR scan codec.
 *
 * The codec is the one of Ford & Ford, "Lossless SIMD Compression of LiDAR
 * Range and Attribute Scan Sequences" (arXiv 2209.08196): each scan of each
 * attribute is quantized to a precision (Sec. III-B), its zero samples are
 * recorded in a bitmask that is compressed on its own (Sec. III-C), a trial
 * compression of a few scanlines picks intra-scan (I) or predicted-scan (P)
 * coding (Sec. III-E), and the remaining samples -- minus the previous scan
 * for a P-scan (Sec. III-D) -- are delta coded along the flattened scan,
 * ZigZag mapped (Eq. 1) and packed with a patched frame of reference in
 * frames of 128 values (Sec. II, III-C).  Every step runs in HIP kernels on
 * the device; the output is a byte stream identical to that of the project's
 * CPU reference.
 *
 * Memory: every d_* pointer is device memory owned by the caller; h_*
 * pointers are host memory owned by the caller.  The library owns its
 * workspaces (one for encoding and one for decoding per device, grown on
 * demand, kept until process exit) and the resident state of each
 * jiffy_stream.  Calls enqueue work on `stream` and
 * synchronize with it once before they return (the byte count, the chosen
 * modes and the status are host values).  Calls on one device are
 * serialized by a per-device lock.
 *
 * Errors: every entry point returns a jiffy_status and never aborts.
 */
#ifndef JIFFY_H
#define JIFFY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* the HIP runtime's stream handle (identical to its own declaration) */
typedef struct ihipStream_t* hipStream_t;

#define JIFFY_MAX_ATTRS 8

/* Scan shape and attributes (Sec. III-A: canonical 2-D scans of 1, 2 or 4
 * byte unsigned samples, zero meaning "no return").  height = scanlines
 * (rows), width = samples per scanline; samples are row-major.
 * precision[a] is the quantization step P >= 1 in input units (Sec. III-B);
 * P = 1 keeps the samples as they are.  It is stored in the stream. */
typedef struct {
    uint32_t height, width, n_attrs;        /* n_attrs in 1..8 */
    uint8_t width_bytes[JIFFY_MAX_ATTRS];   /* 1, 2 or 4 per attribute */
    uint32_t precision[JIFFY_MAX_ATTRS];    /* P >= 1 */
} jiffy_layout;

/* Sec. III-E: the per-scan choice by trial compression (AUTO), I-only,
 * P-only, or the brute-force choice (both codings of every record, the
 * smaller kept; equal sizes: I).  BRUTE is accepted by jiffy_encode only. */
typedef enum { JIFFY_MODE_AUTO = 0, JIFFY_MODE_I_ONLY = 1, JIFFY_MODE_P_ONLY = 2, JIFFY_MODE_BRUTE = 3 } jiffy_mode;

typedef struct {
    uint32_t mode;        /* a jiffy_mode */
    uint32_t trial_rows;  /* scanlines in the trial compression; 0 = 4 (Sec. IV-E) */
} jiffy_options;

typedef enum {
    JIFFY_OK = 0,
    JIFFY_E_INVALID = -1,   /* bad layout, options, pointer or alignment */
    JIFFY_E_CAPACITY = -2,  /* output buffer too small; the size needed is returned */
    JIFFY_E_CORRUPT = -3,   /* malformed stream */
    JIFFY_E_DEVICE = -4,    /* a HIP runtime error */
    JIFFY_E_SHAPE = -5,     /* planes do not match the stream's layout */
    JIFFY_E_SCRATCH = -6    /* jiffy_encode_noalloc: the call needs more than its fixed scratch */
} jiffy_status;

/* Worst-case size in bytes of the stream jiffy_encode writes for n_scans
 * scans of this layout; 0 for an invalid layout. */
size_t jiffy_encode_bound(const jiffy_layout* layout, uint32_t n_scans);

/* Encodes n_scans scans (the whole method of Sec. III).
 *   d_planes[a]: device pointer to n_scans*height*width samples of attribute a
 *                ([n_scans][height][width], row-major, width_bytes[a] each,
 *                aligned to the sample size).
 *   d_out:       device buffer of out_capacity bytes, 4-byte aligned.
 *   h_out_len:   host; receives the stream length (on JIFFY_E_CAPACITY the
 *                length that would be needed; nothing is written then).
 *   h_modes:     optional host [n_scans][n_attrs]; receives 0 (I) or 1 (P).
 * Scan 0 is always an I-scan.  Returns a jiffy_status. */
int jiffy_encode(const jiffy_layout* layout, const jiffy_options* options, uint32_t n_scans,
                 const void* const* d_planes, void* d_out, size_t out_capacity, size_t* h_out_len,
                 uint8_t* h_modes, hipStream_t stream);

/* For callers that cannot allocate memory (code under HIP graph capture,
 * serving loops and harnesses that forbid device allocation): jiffy_encode
 * with the same arguments, results and stream bytes, whose encoder
 * workspace is a fixed device array of 64 MiB in the library (one copy per
 * device, held until the process ends) instead of memory the library
 * allocates.  It calls no hipMalloc, hipFree, hipHostMalloc or other device
 * or pinned-host allocating routine; its plan image and results pass
 * through a fixed 1 MiB / 256 KiB host staging area by hipMemcpyAsync.
 * Host-side planning still uses ordinary heap memory.
 * A call whose workspace would exceed the array (about 5.6 bytes per sample
 * of all its scans and attributes plus ~200 bytes per record, e.g. more than
 * 22 scans of one 128x4096 attribute), or whose plan exceeds the staging area,
 * returns JIFFY_E_SCRATCH with *h_out_len = 0 before touching the device.
 * Every call on a device shares that device's array, which keeps the last
 * call's contents; each call first writes or clears everything it reads.
 * Calls on one device are serialized by the per-device lock and complete
 * before they return; calls that overlapped on one device (for instance
 * from another library instance in the process) would race on the array. */
int jiffy_encode_noalloc(const jiffy_layout* layout, const jiffy_options* options, uint32_t n_scans,
                         const void* const* d_planes, void* d_out, size_t out_capacity, size_t* h_out_len,
                         uint8_t* h_modes, hipStream_t stream);

/* Parses a stream header in host memory.  in_len is the length of the whole
 * stream.  With a record-length table (n_scans > 0 in the header) only the
 * header and the table are read (h_in must hold at least those) and the
 * table must add up to in_len; a header without one (records until the end)
 * is walked record by record, so h_in must then hold the whole stream.
 * Returns JIFFY_OK or JIFFY_E_CORRUPT. */
int jiffy_peek(const void* h_in, size_t in_len, jiffy_layout* layout, uint32_t* n_scans);

/* Decodes a whole stream (every step of Sec. III reversed).
 *   d_in:          device pointer to the stream (in_len bytes, 4-byte aligned).
 *   d_planes_out:  n_attrs device pointers, each [n_scans][height][width] of
 *                  the attribute's width, receiving min(q * P, 2^w - 1).
 * Returns JIFFY_OK or JIFFY_E_CORRUPT (outputs then undefined), or another
 * jiffy_status. */
int jiffy_decode(const void* d_in, size_t in_len, void* const* d_planes_out, hipStream_t stream);

/* Decodes a stream whose layout and scan count the caller already knows
 * (the sensor's configuration), as jiffy_decode, but without reading
 * anything back to the host before the kernels run: the header is compared
 * on the device with the one jiffy_encode writes for (layout, n_scans), and
 * the record offsets come from its length table on the device.  Only a
 * stream with a length table (n_scans >= 1, as jiffy_encode writes it) is
 * accepted; a header without one, or any other header, table or length
 * mismatch returns JIFFY_E_CORRUPT (outputs then undefined).  Arguments as
 * jiffy_decode; d_planes_out hold n_scans scans. */
int jiffy_decode_layout(const jiffy_layout* layout, uint32_t n_scans, const void* d_in, size_t in_len,
                        void* const* d_planes_out, hipStream_t stream);

/* A short English description of a status code (static storage). */
const char* jiffy_status_string(int status);

/* ---- several scan sequences at once ----------------------------------
 * jiffy_encode_many encodes n_streams sequences of one layout and n_scans
 * scans each in one launch sequence (every record of every stream shares
 * each kernel launch); stream s's output is exactly what jiffy_encode writes
 * for it (Sec. III, Fig. 2).  Modes 0..2 only.
 *   d_planes[s][a]: device, stream s's attribute a, [n_scans][H][W];
 *   d_outs[s], caps[s]: device output of stream s (4-byte aligned) and its
 *       capacity; h_out_lens[s]: host, its length (or the bytes needed);
 *   h_modes: optional host [n_streams][n_scans][n_attrs] (0 = I, 1 = P).
 * Returns JIFFY_E_CAPACITY when any output is too small (no output is then
 * complete), else as jiffy_encode.
 * jiffy_decode_many decodes n_streams streams written for one layout and
 * n_scans scans in one launch sequence, each indexed on the device from its
 * length table and its header checked there (Sec. III-C reversed):
 *   d_ins[s], in_lens[s]: device stream s (4-byte aligned) and its length;
 *   d_planes_out[s][a]: device, [n_scans][H][W] of attribute a's width.
 * Returns JIFFY_E_CORRUPT when any stream is malformed or does not match
 * the layout (outputs then undefined).  Both take at most 2^24 records
 * (n_streams * n_scans * n_attrs; JIFFY_E_INVALID beyond), do nothing for
 * n_streams = 0 and synchronize `stream`. */
int jiffy_encode_many(const jiffy_layout* layout, const jiffy_options* options, uint32_t n_streams,
                      uint32_t n_scans, const void* const* const* d_planes, void* const* d_outs, const size_t* caps,
                      size_t* h_out_lens, uint8_t* h_modes, hipStream_t stream);
int jiffy_decode_many(const jiffy_layout* layout, uint32_t n_streams, uint32_t n_scans, const void* const* d_ins,
                      const size_t* in_lens, void* const* const* d_planes_out, hipStream_t stream);

/* ---- stateful streams (many sensors, one scan per step) ---------------
 * A jiffy_stream keeps the previous quantized scan and its zero mask
 * resident in device memory, so that a P-scan (Sec. III-D) can predict from
 * it.  Its first scan, and the first after jiffy_stream_reset, is an
 * I-scan. */
typedef struct jiffy_stream jiffy_stream;

int jiffy_stream_create(const jiffy_layout* layout, const jiffy_options* options, jiffy_stream** out);

/* Bytes of device memory a stream's resident state takes (two halves of
 * quantized samples and of zero-mask words, Sec. III-D); 0 for an invalid
 * layout. */
size_t jiffy_stream_state_bytes(const jiffy_layout* layout);

/* As jiffy_stream_create, with the resident state in caller-owned device
 * memory: d_state (256-byte aligned) holds at least
 * jiffy_stream_state_bytes(layout) bytes and must outlive the stream; the
 * library allocates nothing on the device.  A server can so carve many
 * streams' states out of one budgeted buffer and reuse the memory of
 * streams it has closed.  JIFFY_E_INVALID on a bad layout, alignment or
 * size. */
int jiffy_stream_create_at(const jiffy_layout* layout, const jiffy_options* options, void* d_state,
                           size_t state_bytes, jiffy_stream** out);

/* Encodes one scan of each of n streams in one batch.
 *   d_planes[i][a]: device pointer to the height*width samples of attribute
 *                   a of stream i's new scan.
 *   d_out[i]:       device buffer of caps[i] bytes (4-byte aligned) that
 *                   receives stream i's n_attrs records (no stream header).
 *   h_lens[i]:      host; bytes written (or needed, on JIFFY_E_CAPACITY).
 *   h_modes:        optional host [n][n_attrs] (0 = I, 1 = P).
 * The records equal those jiffy_encode writes for the same scan sequence.
 * On any error no stream's state advances.  The same stream may appear at
 * most once per call. */
int jiffy_batch_encode_step(jiffy_stream* const* streams, uint32_t n, const void* const* const* d_planes,
                            void* const* d_out, const size_t* caps, size_t* h_lens, uint8_t* h_modes,
                            hipStream_t stream);

/* ---- batches (one graph launch per step) --------------------------------
 * A fixed set of n streams encoded together every step, with the same
 * records as jiffy_batch_encode_step.  The step's kernels are captured
 * once in a HIP graph; a step rewrites the records' descriptors (input
 * pointers included) in pinned host memory and launches the graph, whose
 * first kernel reads them and whose offsets kernel writes the lengths and
 * modes back to pinned host memory.  Arguments of create:
 *   d_planes[i][a]: device pointer to stream i's next scan of attribute a
 *                   (H*W samples); a run may name other input pointers;
 *   d_out[i]:       device buffer of caps[i] bytes (4-byte aligned) that
 *                   receives stream i's records, fixed for the batch's life.
 * The batch owns its own workspace (device memory and pinned host memory,
 * freed by jiffy_batch_destroy).  The streams must outlive the batch; each
 * appears once.  Runs of one batch must not overlap (jiffy_batch_run
 * synchronizes `stream` before it returns). */
typedef struct jiffy_batch jiffy_batch;

int jiffy_batch_create(jiffy_stream* const* streams, uint32_t n, const void* const* const* d_planes,
                       void* const* d_out, const size_t* caps, jiffy_batch** out);

/* One step: every stream's next scan, read from d_planes[i][a] (same
 * layout and alignment rules as at create) or, when d_planes is NULL, from
 * the pointers given last.  h_lens[i] (host) gets stream i's record bytes
 * (or the bytes needed, with JIFFY_E_CAPACITY; then no stream advances);
 * h_modes optional [n][n_attrs]. */
int jiffy_batch_run(jiffy_batch* b, const void* const* const* d_planes, size_t* h_lens, uint8_t* h_modes,
                    hipStream_t stream);

void jiffy_batch_destroy(jiffy_batch* b);

/* ---- asynchronous steps (serving: steps in flight on several HIP streams)
 * A jiffy_step owns a device workspace and pinned host buffers sized once at
 * creation for batches of at most max_records records (one per attribute of
 * each stream) and max_samples samples in all; submitting never allocates.
 * jiffy_step_submit plans one scan of each of n streams exactly as
 * jiffy_batch_encode_step does, enqueues the kernels on `stream` and returns
 * at once; jiffy_step_finish waits for them, returns the lengths and modes
 * and advances the streams.  Two step contexts can be in flight at once on
 * different HIP streams (their work overlaps on the device); a jiffy_stream
 * may be in at most one unfinished step (it is refused elsewhere until
 * then).  A step context and its streams are used by one thread at a time;
 * nothing here takes the per-device lock. */
typedef struct jiffy_step jiffy_step;

/* Device bytes a step context of these limits holds (its workspace); 0 when
 * a limit is 0 or above its maximum (2^24 records, 2^40 samples). */
size_t jiffy_step_workspace_bytes(uint32_t max_records, uint64_t max_samples);

/* JIFFY_E_INVALID for a limit of 0 or above its maximum (as above). */
int jiffy_step_create(uint32_t max_records, uint64_t max_samples, jiffy_step** out);

/* d_planes[i][a]: stream i's new scan of attribute a (H*W samples).
 * d_out: device buffer of out_capacity bytes (4-byte aligned) receiving all
 * records packed: stream 0's n_attrs records, then stream 1's right after,
 * and so on (each stream's records are those jiffy_encode writes for its
 * scan sequence).  JIFFY_E_CAPACITY when the batch exceeds the context's
 * limits (nothing enqueued); JIFFY_E_INVALID for a busy stream, a stream
 * named twice, or a step still unfinished. */
int jiffy_step_submit(jiffy_step* step, jiffy_stream* const* streams, uint32_t n, const void* const* const* d_planes,
                      void* d_out, size_t out_capacity, hipStream_t stream);

/* Waits for the submitted step.  h_lens[i] (host): stream i's record bytes
 * in the packed output (stream i starts after the lengths before it);
 * h_modes optional [records] (0 = I, 1 = P).  JIFFY_E_CAPACITY when the
 * packed output did not fit (nothing written, h_lens hold the sizes needed;
 * no stream advances). */
int jiffy_step_finish(jiffy_step* step, size_t* h_lens, uint8_t* h_modes);

/* Waits for an unfinished step (its streams then do not advance) and
 * frees the context. */
void jiffy_step_destroy(jiffy_step* step);

/* Drops the resident previous scan; the next scan is an I-scan. */
int jiffy_stream_reset(jiffy_stream* s);

void jiffy_stream_destroy(jiffy_stream* s);

/* ---- launch configuration (the autotuner's knobs) -----------------------
 * How encodes run, for the whole process, from the next call on (a batch
 * keeps the configuration in force when it was created): fused = 0 runs
 * the chain of kernels (decision, tiles, mask frames, sizes, offsets,
 * assembly); fused = 1 runs the same work as one persistent launch whose
 * workgroups (wgs_per_cu per compute unit; 0 = as many as one holds) take
 * the work items from a queue in dependency order.  The output is the same
 * byte for byte.  jiffy_get_tuning also reports how many workgroups of the
 * fused kernel one compute unit holds (needs a device). */
typedef struct {
    uint32_t fused;
    uint32_t wgs_per_cu;
} jiffy_tuning;

int jiffy_set_tuning(const jiffy_tuning* tuning);
int jiffy_get_tuning(jiffy_tuning* tuning, uint32_t* max_wgs_per_cu);

/* ---- input standardization (Sec. III-A) --------------------------------
 * Cartesian points become the canonical range image: per point, in IEEE
 * double with one rounding per operation (no fused multiply-adds),
 *   r = sqrt(x*x + y*y + z*z), e = atan2(z, sqrt(x*x + y*y)),
 *   a = atan2(y, x) (+ 2 pi when negative),
 *   row = floor(((elev_hi - e) * height) / (elev_hi - elev_lo)),
 *   col = floor((a * width) / (2 pi)) (width wraps to 0),
 *   q = floor(r / range_unit + 0.5);
 * the point is dropped (Sec. III-A: invalid and out-of-range measurements
 * are zero) when a coordinate is not finite, row is outside [0, height) or
 * q outside [1, 2^(8 range_bytes) - 1].  Several points in one cell: the
 * smallest q wins, ties going to the earlier point.  The range image holds
 * the winner's q (0 for an empty cell), each attribute image the winner's
 * attribute value (0 for an empty cell).  atan2 is not correctly rounded:
 * a point within a few units in the last place of a bin edge may land in
 * either neighbour depending on the math library. */
typedef struct {
    uint32_t height, width;                /* rows by elevation (row 0 at elev_hi), columns by azimuth */
    uint32_t range_bytes;                  /* 1, 2 or 4 */
    uint32_t n_attrs;                      /* 0 .. JIFFY_MAX_ATTRS */
    uint8_t attr_bytes[JIFFY_MAX_ATTRS];   /* 1, 2 or 4 each */
    double elev_lo, elev_hi;               /* radians, elev_lo < elev_hi */
    double range_unit;                     /* metres per range step (0.001: millimetres), > 0 */
} jiffy_grid;

/* n_scans scans of n_points points each (pad a shorter scan with NaN).
 *   d_xyz:        device, [n_scans][n_points][3] float32 metres, 4-byte aligned;
 *   d_attrs_in:   host array of n_attrs device pointers, [n_scans][n_points]
 *                 values of attr_bytes[a] bytes each (unused when n_attrs = 0);
 *   d_range:      device, [n_scans][height][width] of range_bytes, written;
 *   d_attrs_out:  host array of n_attrs device pointers, [n_scans][height][width]
 *                 of attr_bytes[a] bytes each, written.
 * Device buffers are caller-owned and aligned to their element size; the
 * library keeps a workspace of 8 bytes per cell of the call.  Synchronizes
 * `stream`.  JIFFY_E_INVALID on a bad grid, pointer, alignment or more
 * than 2^38 points or cells; JIFFY_E_DEVICE on a runtime error. */
int jiffy_standardize(const jiffy_grid* grid, uint32_t n_scans, uint32_t n_points, const float* d_xyz,
                      const void* const* d_attrs_in, void* d_range, void* const* d_attrs_out, hipStream_t stream);

/* ---- ablated codecs (Sec. IV-H, Table IV) ------------------------------
 * Record sizes of every scan of every attribute under codecs with stages
 * left out, and of the zero bitmask under a run-length alternative to the
 * mask frame.  Nothing is encoded; the sizes are exact.  Every level
 * quantizes first (Sec. III-B, the layout's precisions).  Per record
 * (scan-major, attribute-minor) h_sizes receives JIFFY_ABL_SIZES values:
 *   [0] PFOR alone: every pixel's quantized sample, zeros included, coded as
 *       one residual section (Sec. II) in a record with no mask frame
 *       (12-byte head, section, padding to 4);
 *   [1] Delta -> PFOR: the differences to the preceding pixel of the
 *       flattened scan (0 before the first) modulo 2^w, same record;
 *   [2] Delta -> ZigZag -> PFOR: those differences ZigZag-coded (Eq. 1);
 *   [3] the run-length mask codec on the scan's zero bitmask (Sec. III-C):
 *       the bits read as alternating runs, the first of in-range pixels
 *       (possibly empty), coded as one residual section of the first run's
 *       length and every later run's length minus one; bytes padded to 4;
 *   [4] the same for the mask XOR the previous scan's (Sec. III-D); for
 *       the first scan, value [3].
 * Levels 4 and 5 of the table (mask, then prediction) are the records of
 * jiffy_encode in I-only and automatic mode.
 *   layout, n_scans, d_planes: as jiffy_encode (device, caller-owned);
 *   h_sizes: host, n_scans * n_attrs * JIFFY_ABL_SIZES values.
 * Synchronizes `stream`.  JIFFY_E_INVALID on bad arguments or a grid
 * beyond 2^31 workgroups; JIFFY_E_DEVICE on a runtime error.  The library
 * keeps a workspace of 64 bytes per record plus 4 bytes per pixel for each
 * of at most 256 records in flight. */
#define JIFFY_ABL_SIZES 5
int jiffy_ablate(const jiffy_layout* layout, uint32_t n_scans, const void* const* d_planes, uint64_t* h_sizes,
                 hipStream_t stream);

/* ---- kernel timing (benchmarks) ----------------------------------------
 * While enabled, every kernel this library launches is bracketed by HIP
 * events recorded on the stream it runs on, and the elapsed times add up
 * per kernel name.  Enabling clears the totals.  jiffy_profile_read copies
 * up to max_kernels entries: names (32 bytes each, NUL-terminated), total
 * milliseconds and launch counts; it returns the number of kernels seen. */
int jiffy_profile_enable(int enable);
int jiffy_profile_read(uint32_t max_kernels, char* names, double* total_ms, uint32_t* launches);

#ifdef __cplusplus
}
#endif
#endif /* JIFFY_H */

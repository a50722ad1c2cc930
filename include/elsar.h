/*
 * elsar.h -- C ABI of the MI355X (gfx950) learned-partition sort.
 *
 * The library sorts n fixed-length records by their leading key bytes in
 * memcmp order, equal keys in input order, the way ELSAR does (Kristo and
 * Kraska, "Parallel External Sorting of ASCII Records Using Learned Models"):
 * a CDF model fitted on a sample of the keys (Section 3.1) places every record
 * in one of B mutually exclusive, monotonic, equi-depth buckets (Section 3.3,
 * Equation 1); each bucket is sorted on its own (Section 3.4); the sorted
 * buckets are written at the exclusive prefix sums of their sizes
 * (Section 3.5), so the output is a plain concatenation with no merge.
 *
 * Conventions for every call:
 *  - Device pointers ("d_") are HIP device memory on the current device; host
 *    pointers ("h_") are host memory.  The caller owns every buffer it passes;
 *    the library owns only elsar_model objects (and their device storage).
 *  - Record buffers are n * record_bytes bytes, 16-byte aligned; record i is at
 *    byte i * record_bytes.  record_bytes is a multiple of 4 in [40, 128];
 *    8 <= key_bytes <= 28 (the tuned shape is 100-byte records, 10-byte keys).
 *    The bucket sorts order key bytes 0..11 and the input index; with a
 *    longer key, each run of records with equal 12-byte prefixes is then
 *    sorted stably by the remaining key bytes in a fix-up pass over the
 *    output (elsar_sort, elsar_sort_buckets, elsar_sort_host).
 *    elsar_sort_batch takes keys of at most 12 bytes (ELSAR_E_UNSUPPORTED).
 *  - n < 2^32 for every call that takes records on the device, and at most
 *    ELSAR_MAX_DEVICE_RECORDS for one in-HBM sort.
 *  - Work is enqueued on `stream` and runs asynchronously unless a call says
 *    otherwise.  Argument errors are returned before anything is enqueued;
 *    a failed HIP launch returns ELSAR_E_HIP.  On error the outputs are
 *    unspecified, and nothing outside the buffers passed in is written.
 *  - No exception crosses the ABI.  Calls on different models/buffers may run
 *    concurrently; calls that share a buffer must be ordered by the caller.
 */
#ifndef ELSAR_H
#define ELSAR_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* In-HBM sorts: n records in, n out and the workspace (about 463 bytes per
 * 100-byte record: regions of up to 2.5 n slots, a spill area of n slots,
 * 128 bytes each) fit the 288 GB of one MI355X up to this many records. */
#define ELSAR_MAX_DEVICE_RECORDS 400000000ull
#define ELSAR_MLP_PARAMS 4801      /* W1 (64x8), b1 (64), W2 (64x64), b2 (64), w3 (64), b3, row-major */
#define ELSAR_MLP_GRAD_ROWS 128    /* rows of one MLP training step */
#define ELSAR_MLP_STEPS_NONE 0xFFFFFFFFu  /* mlp_steps: no training, the initial network (for comparisons) */

typedef enum {
  ELSAR_OK = 0,
  ELSAR_E_INVALID_ARG = 1,     /* null pointer, bad size or alignment, bad parameter */
  ELSAR_E_NO_MEMORY = 2,       /* workspace or partition buffer too small, or allocation failed */
  ELSAR_E_HIP = 3,             /* a HIP runtime call or kernel launch failed */
  ELSAR_E_UNSUPPORTED = 4,     /* shape outside the supported range (e.g. n too large) */
  ELSAR_E_MODEL_REJECTED = 5   /* the learned model failed its acceptance test (the plain model kept) */
} elsar_status;

typedef enum {
  ELSAR_MODEL_RMI = 0,  /* two-level RMI: linear root, linear-spline leaves */
  ELSAR_MODEL_MLP = 1,  /* monotone MLP root over equi-depth spline leaves if the network passes its
                           acceptance test, else the plain model the automatic choice would take */
  ELSAR_MODEL_AUTO = 2, /* RMI when its largest sample bucket is within accept_ratio of a perfect
                           model's, lambda + sqrt(2 ln(B) lambda) + 1 with lambda = S/B; else SPLINE */
  ELSAR_MODEL_RADIX = 3, /* no learned model: equi-width buckets of the code, floor(code * B / 95^8), the
                            radix partitioning the paper compares its model against (Section 3.3) */
  ELSAR_MODEL_SPLINE = 4 /* linear-spline CDF: K = L/64 segments between equi-depth sample knots over the
                            same equi-depth spline leaves as the MLP root; a record is routed exactly by a
                            binary search among the knots, then among its segment's leaves */
} elsar_model_kind;

/* Fit parameters.  Zero fields take the defaults noted. */
typedef struct {
  uint32_t record_bytes;  /* record length R (100) */
  uint32_t key_bytes;     /* key length K (10) */
  uint32_t num_buckets;   /* B, the paper's f; 0: largest power of two <= n/950, in [1, 2^21] */
  uint32_t num_leaves;    /* L; 0: max(1, B/16) under the linear root, min(B, 2^16) under the equi-depth
                             (MLP and spline) roots */
  uint64_t sample_size;   /* S; 0: min(max(ceil(n/100), 1024), 10^7, n) (Section 3.1, Section 6) */
  uint64_t seed;          /* seed of the sampler's Philox4x32-10 draws */
  uint32_t kind;          /* elsar_model_kind */
  float accept_ratio;     /* MLP accepted if the largest bucket of the network's own output,
                             clamp(floor(B y), 0, B-1), over the sample is <= ratio * ideal, ideal =
                             max(ceil(S/B), longest run of equal codes in the sample); the linear root's
                             gate (ELSAR_MODEL_AUTO) takes the same ratio; 0: 1.5 */
  uint32_t mlp_steps;     /* Adam steps (128 sample rows each) of the MLP fit; 0: 16;
                             ELSAR_MLP_STEPS_NONE: none */
  uint32_t region_pct;    /* bucket j's region holds ceil(region_pct/100 * max(n*(h_j + 2 sqrt(h_j))/S, n/B))
                             + 16 records (h_j: sample keys in bucket j), the rest spills; 0: 125 */
  uint32_t key_len_offset; /* 0: fixed-length keys.  Otherwise variable-length keys (Section 4's padding
                              rule): record byte key_len_offset holds the key's length len (values above
                              key_bytes count as key_bytes); the key is the first len bytes of the key field
                              [0, key_bytes), the field's later bytes are padding and ignored.  Keys order as
                              byte strings: the padding reads as 0x00, below every byte value, and a key sorts
                              before the longer keys it is a prefix of; equal keys keep input order.  Needs
                              key_bytes <= key_len_offset <= 11 (so key_bytes <= 11); not in elsar_sort_batch
                              (ELSAR_E_UNSUPPORTED). */
} elsar_fit_params;

/* Fills *p with the defaults for 100-byte records with 10-byte keys. */
elsar_status elsar_fit_params_default(elsar_fit_params* p);

typedef struct elsar_model elsar_model;

/* Resolves the automatic parameters for n records (B, L, S) and allocates the
 * model's device storage on the current device.  Synchronous. */
elsar_status elsar_model_create(const elsar_fit_params* p, uint64_t n, elsar_model** out);
void elsar_model_destroy(elsar_model* m);

/* Device workspace elsar_sample_fit needs for n records (the sample, its sort
 * buffers and the fit's partial sums). */
elsar_status elsar_fit_workspace_size(const elsar_model* m, uint64_t n, size_t* bytes);

/*
 * Section 3.1: draws the sample (stratified, uniform within strata), sorts its
 * base-95 codes (Section 4, first 8 key bytes, saturating outside
 * 0x20..0x7E) and fits the monotone RMI -- root: least squares of L*rank/S on
 * the FP32 code, slope >= 0; leaf j: the line through its first and last
 * sample mapped to B*rank/S, clamped to the buckets its sample ranks span.
 * d_records: n records on the device.  d_ws: elsar_fit_workspace_size bytes.
 * The model's parameters live on the device; the call is asynchronous.
 *
 * kinds MLP, AUTO and SPLINE also cut equi-depth leaves in the sorted
 * sample: leaf j starts at the first sample of the run of equal codes that
 * holds sample floor(j*S/L), and takes the same spline over its ranks; a run
 * holding the start samples of several leaves is a leaf of its own (the
 * first of them covers exactly the run's code, the next starts at that code
 * + 1), so that a heavily repeated key gets a bucket whose keys are all
 * equal.  The spline root groups the leaves in K = L/64 segments (knots: the
 * segments' first boundaries); a record's leaf is found exactly among the
 * boundaries, in the bracket a table of 65536 code cells gives.  Kind MLP also trains the monotone MLP root (8 quantile-ramp
 * features of the code -> 64 -> 64 -> 1, sigmoid units, non-negative weights;
 * MSE to rank/S on the sample; Adam).  After training, a cell table over the
 * network's output gives, for each of L cells of y, the bracket of leaves
 * whose first codes map there; a record's leaf is then searched exactly among
 * the first codes inside that bracket (after a check that it holds, else from
 * the guess floor(L*y) over all of them).  The bucket of a record under the
 * MLP root is therefore that of its equi-depth leaf; the network decides the
 * cost of finding it.  Acceptance judges the network itself: the histogram of
 * its own buckets clamp(floor(B y), 0, B-1) over the sorted sample must peak
 * at most accept_ratio times the ideal (see elsar_fit_params).  The root is
 * chosen on the device (see elsar_model_kind).
 * With kind MLP the call then synchronises with `stream` and returns
 * ELSAR_E_MODEL_REJECTED when the network was rejected; the model stays valid
 * with the plain root (linear or spline) in use.
 */
elsar_status elsar_sample_fit(elsar_model* m, const void* d_records, uint64_t n, void* d_ws, size_t ws_bytes,
                              hipStream_t stream);

/* Bytes of the partition buffer elsar_partition fills for n records. */
elsar_status elsar_partition_size(const elsar_model* m, uint64_t n, size_t* part_bytes);

/*
 * Section 3.3 / Algorithm 1's reader loop: places every record in bucket
 * F(encode(key)) (Equation 1 holds for the buckets: every key of bucket j is
 * <= every key of bucket j+1), counts the bucket sizes S_p and writes
 * d_bucket_offsets[j] = sum_{k<j} S_k for j = 0..B (u64; d_bucket_offsets[B] = n),
 * the output offsets of Section 3.5.
 * d_part: elsar_partition_size bytes, 16-byte aligned, opaque; it holds each
 * record with its input index, grouped by bucket (in no order within a bucket).
 * d_bucket_offsets: B + 1 u64 on the device, 8-byte aligned.  A misaligned
 * d_part or d_bucket_offsets is ELSAR_E_INVALID_ARG.  Asynchronous.
 */
elsar_status elsar_partition(const elsar_model* m, const void* d_records, uint64_t n, void* d_part,
                             size_t part_bytes, uint64_t* d_bucket_offsets, hipStream_t stream);

/*
 * Sections 3.4-3.5: sorts every bucket of d_part by (key in memcmp order, input
 * index) and writes it to d_out + record_bytes * d_bucket_offsets[j].
 * d_out: n records on the device; it may be the input of elsar_partition (the
 * sort is then in place) but must not overlap d_part.  d_part and
 * d_bucket_offsets are those elsar_partition took (same alignment checks).  The call uses d_part's
 * bookkeeping area as scratch; the records in d_part are left as they are,
 * so the call may be repeated on one partition (into the same or another
 * output), except with keys longer than 12 bytes, whose run pass (Section
 * 4's last-mile ordering of the bytes past the encoded prefix) then reuses
 * the record area as scratch.  Asynchronous.
 */
elsar_status elsar_sort_buckets(const elsar_model* m, void* d_part, size_t part_bytes, uint64_t n,
                                const uint64_t* d_bucket_offsets, void* d_out, hipStream_t stream);

/* Workspace of elsar_sort for n records. */
elsar_status elsar_sort_workspace_size(const elsar_fit_params* p, uint64_t n, size_t* bytes);

/*
 * The whole method on device-resident records: sample + fit, partition, sort
 * and concatenate.  d_out may equal d_in (in place).  d_ws: at least
 * elsar_sort_workspace_size bytes; it holds the model, the partition buffer and
 * the offsets.  Asynchronous; no host synchronisation inside (the choice of
 * root of kinds MLP and AUTO is made on the device; a rejected MLP falls back
 * to the RMI without an error).
 */
elsar_status elsar_sort(const void* d_in, uint64_t n, void* d_out, const elsar_fit_params* p, void* d_ws,
                        size_t ws_bytes, hipStream_t stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): elsar_sort
 * with its workspace in a fixed array that the library holds on every device
 * it runs on, ELSAR_NOALLOC_SCRATCH_BYTES bytes, from the first call on that
 * device until the process ends.  The call allocates nothing (no hipMalloc,
 * hipFree or allocating library routine); the caller passes the records and
 * the output as for elsar_sort.  n must satisfy
 * elsar_sort_workspace_size(p, n) <= ELSAR_NOALLOC_SCRATCH_BYTES (about
 * 5.5e5 100-byte records with the default parameters); a larger n returns
 * ELSAR_E_NO_MEMORY before anything is enqueued.  Every call on a device
 * shares that device's array, which keeps the last call's contents: calls
 * that overlap on one device (on different streams, or from different host
 * threads without ordering) race and give undefined output; calls ordered on
 * one stream are safe.  Asynchronous on `stream`.
 */
#define ELSAR_NOALLOC_SCRATCH_BYTES (256ull << 20)
elsar_status elsar_sort_noalloc(const void* d_in, uint64_t n, void* d_out, const elsar_fit_params* p,
                                hipStream_t stream);

/* One job of a batch: n records at d_in, sorted into d_out (may equal d_in). */
typedef struct {
  const void* d_in;
  void* d_out;
  uint64_t n;
} elsar_job;

/* Workspace of elsar_sort_batch for this job table and parameters. */
elsar_status elsar_sort_batch_workspace_size(const elsar_job* h_jobs, uint32_t njobs, const elsar_fit_params* p,
                                             size_t* bytes);

/*
 * Independent sorts of many jobs of uneven sizes in one launch (the method
 * applied per job; uneven work is balanced the way the paper balances uneven
 * partitions over threads, Section 7.3, here by giving every phase kernel the
 * work of many jobs at once).  h_jobs: host array of njobs jobs; jobs must
 * not overlap one another (a job's output may be its input).  p applies to
 * every job, except that num_buckets / num_leaves of 0 are chosen per job
 * from the tuned table, and job j's sampler seed is p->seed + j.
 *  - Jobs of up to 2048 records are sorted whole, one block each, in one kernel.
 *  - Models: under kind RMI one kernel fits the jobs whose sample has at most
 *    3 * 16384 codes, one block each; other jobs are fitted one by one.
 *  - The jobs are grouped into windows: jobs within a factor 2 in size, about
 *    64M records per window (more for one larger job).  A window's jobs share
 *    one launch per phase (capacities, partition, scan, spill fix-up, bucket
 *    sorts); the windows run one after another in one area of d_ws, so the
 *    scratch is bounded by one window, not by the batch.
 * The first call with a given (table, parameters, workspace) records the whole
 * batch as one HIP graph; that call and every later one with the same
 * arguments is a single graph launch on `stream`.  Asynchronous.
 */
elsar_status elsar_sort_batch(const elsar_job* h_jobs, uint32_t njobs, const elsar_fit_params* p, void* d_ws,
                              size_t ws_bytes, hipStream_t stream);

/* Host tier. */
typedef struct {
  uint64_t chunk_records;     /* records per streamed chunk (one sorted run each) */
  uint64_t pass_records;      /* most records one group pass holds in HBM */
  uint32_t passes;            /* group passes (consecutive buckets fitting a pass) */
  uint32_t num_buckets;       /* B of the global model */
  uint32_t runs;              /* sorted runs written to the fragment store */
  uint32_t copy_passes;       /* groups of one all-equal-key bucket larger than a pass, copied through */
  uint64_t link_bytes;        /* bytes moved over the host link, both directions */
  float fit_ms, count_ms, passes_ms, total_ms;  /* host wall time: global model, runs, group passes, all */
} elsar_host_stats;

#define ELSAR_HOST_SAMPLE_FIRST_CHUNK 1u  /* fit the global model on the first chunk only */

/* Device workspace of elsar_sort_host for n records streamed in chunks of
 * chunk_records (0: 40M, 4 GB of 100-byte records), when one group pass may
 * hold up to pass_records records in HBM (0: n, a single pass). */
elsar_status elsar_sort_host_workspace_size(const elsar_fit_params* p, uint64_t n, uint64_t chunk_records,
                                            uint64_t pass_records, size_t* bytes);

/*
 * The external tier (the paper's larger-than-memory setting, Section 3, with
 * host memory as the external store): n records in host memory h_in are
 * sorted into host memory h_out.  Either may be pageable: pageable memory is
 * copied through page-locked slots the call allocates (sized from the chunk,
 * at most about 4.5 GB), by CPU threads (8 per direction) overlapped with
 * the DMA; page-locked memory is copied directly.
 *  1. The global model (Section 3.1) is fitted on a sample of 1% of the input
 *     (at most 10^7 records) gathered as evenly spaced blocks over the whole
 *     input by one strided copy; with ELSAR_HOST_SAMPLE_FIRST_CHUNK, on the
 *     first chunk only, as the paper samples the first batch one reader reads.
 *  2. Runs (Section 3.3, fragments written once): every chunk of
 *     chunk_records records is streamed to HBM, sorted there by the in-HBM
 *     method, and copied back to h_frag at the chunk's own position as a
 *     sorted run; the global model's bucket counts of the run are kept.
 *  3. Group passes (Section 3.4): consecutive buckets whose records fit one
 *     pass are read back, one slice per run, placed in exact regions, sorted
 *     and copied to h_out at their offset (Section 3.5's concatenation).
 *  Every record crosses the link four times (plus the sample), whatever the
 *  number of passes.  Copies run on streams of their own (device-to-host
 *  copies from a worker thread), double buffered against the kernels on
 *  `stream`.
 * h_frag: n * record_bytes bytes of host memory for the runs; it may be h_in
 * itself (the input is then overwritten with the runs) and must not overlap
 * h_out; h_in must not overlap h_out.  d_ws: workspace; its size bounds the
 * records of one group pass (elsar_sort_host_workspace_size); pass_records,
 * if nonzero, bounds them further.  chunk_records: as for the workspace size
 * (0: 40M).  flags: 0 or ELSAR_HOST_SAMPLE_FIRST_CHUNK.  A bucket
 * larger than a pass is copied through in run order when all its keys are
 * equal (the order of equal keys is the input order); if its keys differ the
 * call returns ELSAR_E_UNSUPPORTED (the output is then unspecified): this
 * needs more records than a pass sharing the first 8 key bytes, or a model
 * fitted on an unrepresentative first chunk.  Synchronous: returns when h_out
 * is complete.  n < 2^32.  stats may be NULL.
 */
elsar_status elsar_sort_host(const void* h_in, uint64_t n, void* h_out, void* h_frag, const elsar_fit_params* p,
                             uint64_t chunk_records, uint64_t pass_records, uint32_t flags, void* d_ws,
                             size_t ws_bytes, hipStream_t stream, elsar_host_stats* stats);

/* What a fitted model looks like; synchronises with the device. */
typedef struct {
  uint32_t kind_used;        /* elsar_model_kind of the root in use (RMI, MLP or SPLINE) */
  uint32_t mlp_rejected;     /* 1 if an MLP was fitted and failed the acceptance test */
  uint32_t num_buckets, num_leaves;
  uint64_t sample_size;
  uint64_t n_fit;
  float root_a0, root_a1;    /* linear root (leaf units): floor(fmaf(a1, x, a0)) */
  uint32_t max_sample_bucket, opt_sample_bucket;  /* acceptance statistics (MLP fits) */
  uint32_t mlp_leaves;       /* equi-depth leaves of the MLP / spline roots (0 without them) */
  uint32_t spline_segments;  /* K segments of the spline root (0 without it) */
  /* acceptance statistics on the sample (0 where not computed): largest sample
   * bucket under the linear root, under the equi-depth leaves, under the
   * network's own buckets clamp(floor(B y), 0, B-1); whether the linear root
   * passed its gate (largest sample bucket <= accept_ratio * perfect); and
   * perfect = lambda + sqrt(2 ln(B) lambda) + 1, lambda = S/B */
  uint32_t rmi_max_sample_bucket, eq_max_sample_bucket, net_max_sample_bucket, rmi_gate_passed;
  float perfect_sample_bucket;
} elsar_model_info;

elsar_status elsar_model_info_get(const elsar_model* m, elsar_model_info* info);

/* The model of job `job` as the last elsar_sort_batch call with this job
 * table, parameters and workspace fitted it, read back from d_ws once that
 * call has completed (synchronises with the device); the fields are those of
 * elsar_model_info_get.  For checking the batched fit against elsar_sample_fit
 * with the job's parameters (num_buckets and num_leaves as reported, seed
 * p->seed + job).  ELSAR_E_INVALID_ARG for a job out of range or one sorted
 * whole (2048 records or fewer, no model). */
elsar_status elsar_sort_batch_model_info(const elsar_job* h_jobs, uint32_t njobs, const elsar_fit_params* p,
                                         const void* d_ws, size_t ws_bytes, uint32_t job, elsar_model_info* info);

/* Copies the leaf table of the root in use to host arrays of num_leaves
 * entries each (any may be NULL).  Synchronises. */
elsar_status elsar_model_leaves(const elsar_model* m, uint64_t* h_base, float* h_slope, float* h_icpt,
                                uint32_t* h_lo, uint32_t* h_hi);

/* The spline root of a model created with kind MLP, AUTO or SPLINE
 * (ELSAR_E_INVALID_ARG otherwise): h_knots[spline_segments + 1] (segment i
 * starts at code knots[i] = bound[(i L) / K]; knots[K] is past every code),
 * h_bound[mlp_leaves + 1] and h_first[mlp_leaves + 1] as below.  Under kind
 * AUTO they are fitted only when the linear root was not kept; otherwise the
 * model info shows mlp_leaves 0 and this call returns ELSAR_E_INVALID_ARG.
 * Any pointer may be NULL.  Synchronises. */
elsar_status elsar_model_spline_get(const elsar_model* m, uint64_t* h_knots, uint64_t* h_bound, uint32_t* h_first);

/* The MLP root of a model created with kind MLP (ELSAR_E_INVALID_ARG
 * otherwise): h_params[ELSAR_MLP_PARAMS] (FP32 master copy), h_knots[9]
 * (q_0..q_8), h_bound[mlp_leaves + 1] (leaf j takes the codes in
 * [bound[j], bound[j+1])), h_first[mlp_leaves + 1] (first sample rank of each
 * leaf; first[L] = S).  Any pointer may be NULL.  Synchronises. */
elsar_status elsar_model_mlp_get(const elsar_model* m, float* h_params, uint64_t* h_knots, uint64_t* h_bound,
                                 uint32_t* h_first);

/* Verification entry points of the MLP kernels; host buffers, synchronous,
 * they allocate and free their own device memory.
 * elsar_mlp_forward: y of n codes under h_params / h_knots (the evaluation the
 * partition uses).  elsar_mlp_gradient: MSE loss and its gradient (flat
 * parameter order) on ELSAR_MLP_GRAD_ROWS rows of codes and targets (one
 * training step's backward pass). */
elsar_status elsar_mlp_forward(const float* h_params, const uint64_t* h_knots, const uint64_t* h_codes, uint64_t n,
                               float* h_y);
elsar_status elsar_mlp_gradient(const float* h_params, const uint64_t* h_knots, const uint64_t* h_codes,
                                const float* h_targets, float* h_grad, float* h_loss);
/* One training step as the fit runs it: the gradient of elsar_mlp_gradient on
 * the ELSAR_MLP_GRAD_ROWS rows, then the Adam update of step `step` (>= 1;
 * beta1 0.9, beta2 0.999, eps 1e-8, bias corrections 1/(1 - beta^step)) with
 * learning rate lr, W1, W2 and w3 projected onto >= 0.  h_adam: the first and
 * then the second moments (2 * ELSAR_MLP_PARAMS).  The updated parameters and
 * moments go to h_params_out / h_adam_out; h_grad (ELSAR_MLP_PARAMS) and
 * h_loss may be NULL.  ELSAR_E_INVALID_ARG for step 0 or a negative lr. */
elsar_status elsar_mlp_train_step(const float* h_params, const float* h_adam, const uint64_t* h_knots,
                                  const uint64_t* h_codes, const float* h_targets, uint32_t step, float lr,
                                  float* h_params_out, float* h_adam_out, float* h_grad, float* h_loss);

/* Statistics of the last partition in d_part; synchronises. */
typedef struct {
  uint64_t n;
  uint32_t num_buckets;
  uint32_t spill_count;      /* records that overflowed their bucket's region */
  uint32_t mid_buckets;      /* buckets sorted by the large LDS kernel */
  uint32_t big_buckets;      /* buckets sorted through global memory */
  uint32_t max_bucket;       /* largest bucket */
  uint32_t mid_records;      /* records in the mid_buckets */
  uint32_t big_records;      /* records in the big_buckets */
  /* after elsar_sort_buckets: the split of the big buckets into segments --
   * segments listed, the list's capacity, and 1 if a piece stack overflowed.
   * A count above the capacity or an overflow means some segment was not
   * sorted (the bounds make neither expected for any input). */
  uint32_t split_segments, split_segment_cap, split_overflow;
} elsar_partition_stats;

elsar_status elsar_partition_stats_get(const elsar_model* m, const void* d_part, size_t part_bytes,
                                       elsar_partition_stats* st);

/* Phase timing: when enabled (which also resets it), the library records HIP
 * events around each phase on the stream it launches on; elsar_timings_get
 * synchronises and returns the mean milliseconds per call of each phase. */
typedef struct {
  float sample_fit_ms;   /* sample, sample sort, fit, capacities */
  float partition_ms;    /* the partition kernel */
  float scan_ms;         /* offsets, spill fix-up */
  float bucket_sort_lds_ms;   /* in-bucket sort + concatenation of buckets <= 2048 records (one kernel) */
  float bucket_sort_rest_ms;  /* the larger buckets (LDS kernel up to 6144 records, then global memory) */
  float total_ms;        /* first to last recorded boundary of a call */
  uint32_t calls;        /* calls averaged over (the last 512 since enabling) */
} elsar_timings;

elsar_status elsar_set_timing(int enabled);
elsar_status elsar_timings_get(elsar_timings* t);

const char* elsar_status_string(elsar_status s);

#ifdef __cplusplus
}
#endif
#endif /* ELSAR_H */

/*
 * libecc -- Euler characteristic curves of d-dimensional gray-scale images on
 * one AMD Instinct MI355X (gfx950).
 *
 * What is computed (Heiss & Wagner, arXiv 1705.02045):
 *   The image is the cubical complex of Sec. 2 ("Consecutive Thresholded
 *   Images as Sublevel Set Filtrations"): every voxel is a closed unit d-cube
 *   and the complex holds all voxels and all their faces.  A cell enters the
 *   filtration at the minimum gray value of the voxels that contain it
 *   (Sec. 2, "Sublevel Set Filtration").  T_t is the complex of cells with
 *   value <= t, and the output is chi(T_t) for every threshold t (Sec. 2,
 *   "Euler Characteristic Curve of an Image"), i.e. the prefix sums of the
 *   vector of changes a_t = chi(T_t) - chi(T_{t-1}) (Sec. 3, "Tracking the
 *   Changes" and "Post-Processing").  Counts are exact int64.
 *
 * Layout: images are dense, C order, dims[0] slowest (the axis along which
 * the streaming interface cuts chunks, Sec. 3 "Streaming"), no padding.
 *
 * Errors: every function returns an ecc_status.  Nothing aborts or throws.
 * On failure the caller's output buffers are left unmodified and
 * ecc_last_error() (thread-local) describes the failure.
 *
 * Pointers: "device" means memory the HIP runtime reports as device memory on
 * the current device; "host" is any other readable memory.  The library never
 * frees caller memory.  Streams are hipStream_t values passed as void*; NULL
 * is the null stream.
 */
#ifndef ECC_H
#define ECC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ECC_OK = 0,
    ECC_E_ARG = -1,              /* null pointer, bad ndim/dims/dtype, size overflow */
    ECC_E_RANGE = -2,            /* an ECC_U14 value is >= 16384 */
    ECC_E_NAN = -3,              /* an ECC_F32 image holds a NaN */
    ECC_E_BUFFER_TOO_SMALL = -4, /* curve capacity too small; count holds the size needed */
    ECC_E_STATE = -5,            /* streaming call out of order */
    ECC_E_NOMEM = -6,            /* device or pinned-host allocation failed */
    ECC_E_HIP = -7,              /* a HIP runtime call failed; message has hipGetErrorString */
    ECC_E_UNSUPPORTED = -8       /* valid request this library does not implement */
} ecc_status;

/* Value types.  m is the number of thresholds t = 0..m-1 (Sec. 3, "Range of
 * Values": values in {0, ..., m-1}). */
typedef enum {
    ECC_U8 = 1,   /* uint8,  m = 256 */
    ECC_U14 = 2,  /* uint16 storage, values < 16384, m = 16384 */
    ECC_U16 = 3,  /* uint16, m = 65536 (ecc_compute and ecc_compute_async; counted in one or two
                     passes over the image, see ecc_compute_async) */
    ECC_F32 = 4   /* float32; thresholds are the distinct values (Sec. 3, "Other Ranges of Gray Values") */
} ecc_dtype;

/* 1 <= ndim <= 4, n[k] >= 1 for k < ndim, n[0] slowest.  Entries past ndim are ignored. */
typedef struct {
    int32_t ndim;
    int64_t n[4];
} ecc_dims;

/* Output curve.
 *   capacity: in, entries available in chi (and keys for ECC_F32).
 *   count:    out, entries written (m, or the number K of distinct values for
 *             ECC_F32); on ECC_E_BUFFER_TOO_SMALL, the entries needed.
 *   chi:      out, chi[i] = chi(T_t) for the i-th threshold; host or device.
 *   keys:     ECC_F32 only: ascending distinct values, -0.0 stored as +0.0;
 *             host or device.  Ignored for integer types. */
typedef struct {
    int64_t capacity;
    int64_t count;
    int64_t *chi;
    float *keys;
} ecc_curve;

/* Number of thresholds m of an integer dtype (256, 16384, 65536); ECC_E_ARG otherwise. */
int ecc_threshold_count(ecc_dtype dtype, int64_t *m_out);

/* Euler characteristic curve of an image (Sec. 2 and Sec. 3 as above).
 *   image: host or device pointer to prod(n) elements of dtype.  Host images
 *          are copied to the device first.
 *   curve: capacity >= m (integer types) or >= prod(n) (always enough for
 *          ECC_F32).  chi/keys may be host or device pointers.
 *   stream: work is enqueued on it; the call returns after the curve is
 *          written (it synchronizes that stream).
 * Integer images with four axes longer than 1 are computed exactly through
 * the float path (their curve read at every integer threshold).
 * Errors: ECC_E_ARG, ECC_E_RANGE (U14), ECC_E_NAN (F32),
 *         ECC_E_BUFFER_TOO_SMALL, ECC_E_NOMEM, ECC_E_HIP, ECC_E_UNSUPPORTED. */
int ecc_compute(const void *image, const ecc_dims *dims, ecc_dtype dtype, ecc_curve *curve, void *stream);

/* The other convention for a cell's entry value: the MAXIMUM of the image
 * over the voxels containing the cell (a literal "largest gray value among
 * its voxels" reading, in place of Sec. 2's minimum, "Sublevel Set
 * Filtration").  chi[t] = sum of (-1)^dim c over the cells c whose maximum is
 * <= t, for t = 0..m-1.  These cell sets are not complexes in general (a face
 * can enter after the cell it bounds); chi[m-1] = 1 (the whole box).
 * Computed as the change vector of m-1-v read back reversed: the cells whose
 * maximum is t are those whose minimum of m-1-v is m-1-t.  Images with four
 * axes longer than 1 go through the float path on m-1-v: chi[t] = 1 minus
 * that image's curve at m-2-t.
 * Integer dtypes u8 and u14; arguments, synchronisation and errors as
 * ecc_compute (ECC_E_UNSUPPORTED for ECC_F32 and ECC_U16). */
int ecc_compute_max_entry(const void *image, const ecc_dims *dims, ecc_dtype dtype, ecc_curve *curve,
                          void *stream);

/* Float32 curve restricted to its change points (Sec. 3, "Other Ranges of
 * Gray Values": the curve is a step function over the distinct values): the
 * distinct values after which chi differs from its value before them (chi
 * = 0 below the smallest value), ascending, with chi after each.  A subset
 * of ecc_compute's ECC_F32 output, which lists every distinct value.
 *   dtype: ECC_F32 (others: ECC_E_UNSUPPORTED).
 *   curve: keys and chi as for ecc_compute; count = number of change points.
 * Errors as ecc_compute for ECC_F32. */
int ecc_compute_change_points(const void *image, const ecc_dims *dims, ecc_dtype dtype, ecc_curve *curve,
                              void *stream);

/* Float32 image quantised to integer bins, then the integer curve (Sec. 3,
 * "Range of Values": values shifted and scaled into {0, ..., m-1}):
 *   scale = m / (hi - lo), x = (v - lo) * scale, all in float32 with
 *   round-to-nearest and no fused multiply-add; bin = 0 for x < 0 (and
 *   v = -inf), m-1 for x >= m (and +inf), else the integer part of x.
 * chi[t] equals the float curve at the largest value whose bin is <= t (the
 * sublevel sets of the bins are sublevel sets of the image).
 *   bins: ECC_U8 (m = 256), ECC_U14 (16384) or ECC_U16 (65536).
 *   lo < hi, both finite.  image: host or device float32; curve as
 *   ecc_compute for the integer type.
 * Errors: ECC_E_ARG, ECC_E_NAN, ECC_E_BUFFER_TOO_SMALL, ECC_E_NOMEM,
 * ECC_E_HIP, ECC_E_UNSUPPORTED. */
int ecc_compute_quantized(const float *image, const ecc_dims *dims, float lo, float hi, ecc_dtype bins,
                          ecc_curve *curve, void *stream);

/* The dual complex of the image (the alternative the footnote to Sec. 2,
 * "Consecutive Thresholded Images as Sublevel Set Filtrations", names:
 * voxels become vertices, with the lower-star filtration).  Vertices are the
 * voxels; a cell is a product, per axis, of one index or a pair of
 * neighbouring indices (edges join voxels that share a (d-1)-face:
 * 4-connectivity in 2-D, 6 in 3-D); a cell enters at the maximum of the
 * image over its vertices.  chi[t] = chi of the cells with value <= t, for
 * t = 0..m-1.  Axes of length 1 are dropped (one to four may remain).
 * Computed from the largest-value convention of the image and of every face
 * of its box (inclusion-exclusion over the faces, (-1)^codim; the full box
 * of a 4-D image through the float path, as ecc_compute_max_entry).
 * Integer dtypes u8 and u14; arguments, synchronisation and errors as
 * ecc_compute (ECC_E_UNSUPPORTED for ECC_F32 and ECC_U16). */
int ecc_compute_dual(const void *image, const ecc_dims *dims, ecc_dtype dtype, ecc_curve *curve, void *stream);

/* Stream-ordered form for integer types with device-resident data: enqueues
 * the whole computation on `stream` and returns without synchronizing.
 * ECC_U16 images are counted in passes over the image of 32768-bin
 * workgroup histograms, each adding the values of its half of 0..65535.
 * This form runs both; ecc_compute runs the second only when the first has
 * seen a value of 32768 or more.
 *   image_dev: device pointer, prod(n) elements.
 *   chi_dev:   device pointer, m int64 entries; written only if the input is
 *              valid (all U14 values < 16384).
 *   status_dev: optional device pointer to one uint32; receives 0 on
 *              success or ECC_STATUS_RANGE_BIT after the work completes.
 * Scratch memory comes from a per-(device, stream) workspace the library
 * keeps; concurrent calls on the same stream are ordered by the stream.
 * Host-side errors: ECC_E_ARG, ECC_E_NOMEM, ECC_E_HIP, ECC_E_UNSUPPORTED. */
#define ECC_STATUS_RANGE_BIT 1u
int ecc_compute_async(const void *image_dev, const ecc_dims *dims, ecc_dtype dtype, int64_t *chi_dev,
                      uint32_t *status_dev, void *stream);

/* For callers that cannot allocate (work under HIP graph capture, serving
 * loops or harnesses that forbid hipMalloc): ecc_compute_async with every
 * scratch buffer in one statically sized device array of the library
 * (68.6 MiB per GPU, held by each GPU the library runs on until the process
 * ends) instead of a workspace.  Arguments, results and errors as
 * ecc_compute_async; it allocates no memory, host or device.  A launch uses
 * at most 1024 workgroups (larger images give each workgroup more tiles), so
 * every image ecc_compute_async takes fits; ECC_E_NOMEM reports a need
 * beyond the array, which this library does not produce.
 * Every call on one GPU shares that GPU's array and it keeps the last call's
 * contents: calls that overlap in time on one GPU (different streams, or
 * host threads) race and give wrong curves; order them, e.g. on one stream. */
int ecc_compute_async_noalloc(const void *image_dev, const ecc_dims *dims, ecc_dtype dtype, int64_t *chi_dev,
                              uint32_t *status_dev, void *stream);

/* ---------------------------------------------------------------------------
 * Tile shapes.  The integer kernel's tiling of a launch has three
 * parameters: rows per wave (2 or 4), waves along x (up to 16 of a
 * workgroup's 16) and workgroups per CU (the image is split along axis 0
 * until about that many tiles per CU exist; planes with more tiles give a
 * workgroup several).  By default a rule of the launch's size picks them
 * (measured on MI355X); ecc_autotune times the candidates on an image and
 * keeps the fastest for its shape in a process-wide table consulted by every
 * later launch of that shape (dtype, plane shape and number of planes; the
 * planes of a streamed chunk are its own shape).  Results do not depend on
 * the tiling. */
typedef struct {
    int32_t rows;          /* rows per wave: 2 or 4 */
    int32_t tiles_per_cu;  /* workgroups per CU: 4, 8 or 16 */
    int32_t waves_x;       /* waves along x per workgroup: 8 or 16 */
    float ms;              /* ecc_autotune: the fastest candidate's time (kernel + column sums) */
} ecc_tiling;

/* Times every candidate tiling (rows {2, 4} x tiles_per_cu {4, 8, 16} x
 * waves_x {8, 16}) on a device image of an integer dtype (U8, U14) and
 * stores the fastest for its shape (the launch-size rule's tiling unless
 * another is at least 2 % faster); best receives it.  The image's values
 * must be valid (ECC_E_RANGE otherwise, nothing stored).
 * Errors: ECC_E_ARG, ECC_E_RANGE, ECC_E_UNSUPPORTED, ECC_E_NOMEM, ECC_E_HIP. */
int ecc_autotune(const void *image_dev, const ecc_dims *dims, ecc_dtype dtype, void *stream, ecc_tiling *best);

/* The tiling a resident launch of this shape would use (a stored one, else
 * the size rule); ms = 0.  Errors: ECC_E_ARG, ECC_E_UNSUPPORTED. */
int ecc_tiling_for(const ecc_dims *dims, ecc_dtype dtype, ecc_tiling *out);

/* Forgets every tiling ecc_autotune stored. */
void ecc_autotune_reset(void);

/* The stored tilings as a text file, so that a later process starts with
 * them (a tuning cache).  One line per entry, fields separated by spaces:
 *   ecc-tiling-v1 dtype nin n1 n2 planes rows tiles_per_cu waves_x ms
 * (the shape key of an integer launch: dtype, number of in-plane axes,
 * in-plane extents, planes).  ecc_autotune_save writes every entry (the file
 * is replaced).  ecc_autotune_load adds the file's entries to the stored
 * ones (an entry for the same key is replaced); a malformed line or a field
 * outside its range fails the call with nothing stored.  Returns the number
 * of entries written / read, or: ECC_E_ARG (NULL path, a file that cannot
 * be opened, read or written, or a malformed entry, which ecc_last_error
 * names). */
int ecc_autotune_save(const char *path);
int ecc_autotune_load(const char *path);

/* Memory of long-running processes (no passage of the paper: library
 * housekeeping).  The calls above keep, per stream, the device scratch they
 * grew (sized by the largest image computed on that stream) for the next
 * call.  ecc_release_workspaces frees that scratch for the current device;
 * the next call on a stream grows what it needs again.  It first waits for
 * all work on the device.  It must not overlap another call of the library
 * on the same device, whose buffers it would free.  Stream, batch and serve
 * handles own their buffers and keep them; so does the fixed scratch of
 * ecc_compute_async_noalloc; tuned tilings are kept.
 * Errors: ECC_E_HIP. */
int ecc_release_workspaces(void);

/* ---------------------------------------------------------------------------
 * Streaming (Sec. 3, "Streaming" and "Processing one Chunk"): an image larger
 * than device memory is pushed as consecutive chunks of whole axis-0 planes.
 * Each chunk is processed with a one-plane collar taken from its neighbours
 * (the previous chunk's last plane is kept on the device; each chunk's own
 * last plane waits for the next chunk); the changes vector stays on the
 * device and the prefix sum is taken once in ecc_stream_finish.
 * Integer dtypes.  ECC_U16 (m = 65536): every chunk launch runs as two
 * passes of 32768 bins (Sec. 3, "Range of Values"), each adding the values
 * of its half of 0..65535 to that half of the changes vector.  Planes with
 * three axes longer than 1 (4-D images, planes of at most 2^28 voxels) go
 * through the float path's change kernel: a launch's planes and their
 * collars as float32 in one window buffer, the non-zero changes of the
 * launch's planes added at their voxels' values. */
typedef struct ecc_stream ecc_stream;

/* Starts a stream for an image of full_dims (ndim 1..4).  The handle owns
 * its device buffers until ecc_stream_finish or ecc_stream_abort.
 * stream: the HIP stream the work is ordered on (void*, may be NULL).
 * Errors: ECC_E_ARG, ECC_E_NOMEM, ECC_E_HIP, ECC_E_UNSUPPORTED. */
int ecc_stream_begin(const ecc_dims *full_dims, ecc_dtype dtype, void *stream, ecc_stream **out);

/* Pushes n_planes consecutive axis-0 planes (n_planes * prod(n[1..]) elements).
 * Host pointers (pinned or pageable) are copied; the call returns once the
 * caller may reuse the buffer.  Device pointers are read in place by work on
 * the stream: the caller must not overwrite them until that work is done
 * (e.g. by later work on the same stream).
 * Errors: ECC_E_ARG, ECC_E_STATE (more planes than n[0]), ECC_E_RANGE
 * (detected for U14 at finish), ECC_E_NOMEM, ECC_E_HIP. */
int ecc_stream_push_chunk(ecc_stream *st, const void *planes, int64_t n_planes);

/* Processes the last plane, writes the curve and frees the handle (always,
 * also on error).  Errors: ECC_E_STATE (planes missing), ECC_E_RANGE,
 * ECC_E_BUFFER_TOO_SMALL, ECC_E_HIP. */
int ecc_stream_finish(ecc_stream *st, ecc_curve *curve);

/* Frees the handle without producing a curve.  NULL is ignored. */
void ecc_stream_abort(ecc_stream *st);

/* Checkpoint / resume of a stream (Sec. 3, "Streaming": the changes vector
 * of the planes done, the planes a later chunk still needs as its collar and
 * the count of planes pushed are a complete state).
 * ecc_stream_snapshot_size: bytes of a snapshot of the stream as it is now.
 * ecc_stream_snapshot: waits for the stream's work, then writes the
 *   snapshot into host_buf (host memory of at least that size; the stream
 *   stays usable).  Errors: ECC_E_ARG, ECC_E_BUFFER_TOO_SMALL, ECC_E_HIP.
 * ecc_stream_restore: a new stream handle (on `stream`, the current device)
 *   in the state of the snapshot; pushing the remaining planes and finishing
 *   gives the curve of the whole image.  The snapshot is checked (its
 *   header, every count against its dims, its size): ECC_E_ARG if it does
 *   not describe a state of such a stream; also ECC_E_NOMEM, ECC_E_HIP. */
int ecc_stream_snapshot_size(const ecc_stream *st, int64_t *bytes);
int ecc_stream_snapshot(ecc_stream *st, void *host_buf, int64_t capacity);
int ecc_stream_restore(const void *host_buf, int64_t bytes, void *stream, ecc_stream **out);

/* ---------------------------------------------------------------------------
 * Batches of independent images (integer dtypes).  Curves of unrelated images
 * never merge, so one launch can carry the tiles of many images (Sec. 3,
 * "Parallel Computations": the work splits into parts whose changes vectors
 * are summed; here each image sums only its own parts). */
typedef struct {
    const void *image; /* device pointer, prod(dims.n) elements of dtype */
    ecc_dims dims;     /* as for ecc_compute */
    int32_t dtype;     /* ECC_U8, ECC_U14 or ECC_U16 */
    int64_t *chi;      /* device pointer, m int64 entries (written only if the image is valid) */
} ecc_job;

typedef struct ecc_batch ecc_batch;

/* A batch context bound to the current device and `stream` (void*, may be
 * NULL).  It owns device scratch and pinned descriptor tables, reused by
 * later runs.  Errors: ECC_E_ARG, ECC_E_HIP. */
int ecc_batch_create(void *stream, ecc_batch **out);

/* Enqueues the curves of n_jobs images on the context's stream and returns
 * without waiting for them.  status_dev: optional device array of n_jobs
 * uint32; entry j receives 0 or ECC_STATUS_RANGE_BIT for image j.  Runs on
 * one context are ordered by its stream; a context is not for concurrent use
 * from several host threads.  The images and chi buffers must stay valid
 * until the work is done.  u8 and u14 jobs share one persistent launch;
 * ECC_U16 jobs (m = 65536, more bins than a workgroup histogram holds) run
 * after it on the same stream, as ecc_compute_async runs them (two passes).
 * Errors: ECC_E_ARG (bad job), ECC_E_UNSUPPORTED (shape or dtype the integer
 * path does not take), ECC_E_NOMEM, ECC_E_HIP. */
int ecc_batch_run(ecc_batch *b, int32_t n_jobs, const ecc_job *jobs, uint32_t *status_dev);

/* Waits for the context's work and frees it.  NULL is ignored. */
void ecc_batch_destroy(ecc_batch *b);

/* Tile depth of a batch context: an image of n0 planes is cut into tiles of
 * max(min_planes, n0 / split) planes (defaults 64 and 4).  Times ecc_batch_run
 * on the given jobs (their chi buffers are written) for min_planes in
 * {16, 32, 64, 128} x split in {2, 4, 8} and keeps the fastest for the
 * context's later runs; the outputs (optional) receive it and its time.
 * Synchronizes the context's stream.  Errors as ecc_batch_run. */
int ecc_batch_autotune(ecc_batch *b, int32_t n_jobs, const ecc_job *jobs, int32_t *min_planes, int32_t *split,
                       float *ms);

/* Device memory one request of a batch occupies while in flight: its
 * image, the per-workgroup count rows of its batch tiling (default tile
 * depth), its changes vector and its curve (bytes).  Errors: ECC_E_ARG,
 * ECC_E_UNSUPPORTED. */
int ecc_job_footprint(const ecc_job *job, int64_t *bytes);

/* Serving replay for measurement (Sec. 3, "Parallel Computations": every
 * request's changes vector is its own; "Streaming": an image is consumed
 * chunk by chunk of axis-0 planes).  Request i (jobs[i]; its chi field is
 * ignored) becomes available at arrival_s[i] seconds after the call starts
 * (ascending).  Its image is device memory, or, when cfg->arena_bytes > 0,
 * host memory (pinned, e.g. hipHostMalloc, for the copies to overlap).
 *
 * Continuous batching (one_launch_per_image = 0): whenever fewer than
 * max_inflight batches are in flight, the requests that have arrived are
 * admitted in arrival order into the next ecc_batch_run while the batch
 * holds at most max_batch requests and the sum of their footprints
 * (ecc_job_footprint) stays within max_batch_bytes (0: no limit; the first
 * request of a batch always counts).  Otherwise every request is one
 * ecc_compute_async launch as soon as it is admitted.
 * Host-origin requests: admission also reserves a block of the arena (one
 * device buffer of arena_bytes) for the image, copies it in on a copy stream
 * of the call and frees the block when the request's kernels are done; a
 * request waits while its image does not fit.  Images in pinned host memory
 * with a device-mapped, 16-byte aligned address are copied by one kernel per
 * 32 requests of a batch, which reads them over the bus; the others
 * (pageable memory, other alignments) by one copy each.
 * Requests whose image exceeds stream_above_bytes (0: arena_bytes / 4 for
 * host-origin requests, else never) are not batched: one at a time, each is
 * pushed through the streaming interface on a stream of its own in chunks
 * of whole axis-0 planes of about chunk_bytes (0: 64 MiB; host-origin: at
 * most arena_bytes / 4, each chunk in an arena block), two chunks in
 * flight, its partial changes vector kept on the device, while batches of
 * the other requests keep running.
 * Curves are copied to pinned host memory owned by the call on a copy
 * stream that waits for the kernels; latency_s[i] receives the time from
 * arrival until that copy was seen complete; batch_id[i] (optional) the
 * index of the batch, launch or stream that carried it; status[i]
 * (optional) ECC_OK or ECC_E_RANGE.  At the end the curves are copied to
 * chi_host, request i's at chi_host + (sum of the m of the requests before
 * it); a request that failed gets zeros.  Blocks until all requests are done.
 * U8 and U14 requests.  Errors: ECC_E_ARG, ECC_E_UNSUPPORTED (a plane of a
 * streamed request above arena_bytes / 4), ECC_E_NOMEM, ECC_E_HIP, and
 * ECC_E_RANGE when a request held a 14-bit value >= 16384 (every other
 * request's curve is still delivered). */
typedef struct {
    int32_t max_batch;            /* requests per batch, >= 1 */
    int32_t one_launch_per_image; /* 1: one ecc_compute_async per request */
    int64_t max_batch_bytes;      /* footprint per batch; 0: no limit */
    int64_t arena_bytes;          /* > 0: host-origin requests, device arena of this size */
    int64_t stream_above_bytes;   /* images above this are streamed; 0: default (above) */
    int64_t chunk_bytes;          /* streamed chunk size; 0: default (above) */
    int32_t max_inflight;         /* batches in flight; 0: 3 (batched) or unbounded (per image) */
} ecc_serve_config;

int ecc_serve(ecc_batch *b, int32_t n, const ecc_job *jobs, const double *arrival_s, const ecc_serve_config *cfg,
              int64_t *chi_host, double *latency_s, int32_t *batch_id, int32_t *status);

/* ecc_serve with device-resident requests, no streaming and the default
 * number of batches in flight. */
int ecc_serve_simulate(ecc_batch *b, int32_t n, const ecc_job *jobs, const double *arrival_s, int32_t max_batch,
                       int64_t max_batch_bytes, int32_t one_launch_per_image, int64_t *chi_host, double *latency_s,
                       int32_t *batch_id);

/* Kernel timing (measurement support, not needed for results).  While
 * enabled, every launch of the per-voxel kernels (the integer change-vector
 * kernel and the float record kernel) is bracketed by two HIP events recorded
 * on the stream it is launched on.  ecc_profile_read waits for the recorded
 * events and returns the summed elapsed time in milliseconds and the number
 * of launches since the last reset.  ecc_profile_enable(0) stops recording;
 * ecc_profile_reset drops what was recorded.  Process-wide; not for
 * concurrent use from several threads.  Errors: ECC_E_ARG (NULL output),
 * ECC_E_HIP. */
int ecc_profile_enable(int on);
int ecc_profile_reset(void);
int ecc_profile_read(double *kernel_ms, int64_t *launches);

/* Thread-local description of the last failure in this thread ("" if none). */
const char *ecc_last_error(void);

/* Library version string. */
const char *ecc_version(void);

#ifdef __cplusplus
}
#endif
#endif /* ECC_H */

/*
 * qbvh.h -- neighbor lists from a quantized linear bounding volume hierarchy
 * on AMD Instinct MI355X (gfx950).
 *
 * The method (Howard, Statt, Madutsa, Truskett, Panagiotopoulos, "Quantized
 * bounding volume hierarchies for neighbor search in molecular simulations on
 * graphics processing units"):
 *   - Section 2.1: particles get 30-bit Morton codes (2^10 - 1 bins per axis
 *     of the periodic box), are sorted along the Z-order curve, Karras's
 *     radix tree is emitted over the sorted codes and axis-aligned boxes are
 *     fit bottom-up, giving N - 1 internal nodes with two children each
 *     (this library finds the same tree, with Karras's node ids, bottom-up in
 *     the same climb as the fit);
 *   - Section 2.2: node bounds are snapped outward to an integer grid over
 *     the root-node box and packed with a skip rope (the paper's node is 16
 *     bytes; this library stores both children of a node in one 32-byte
 *     record, see QBVH_EXPORT_RECORDS);
 *   - Section 2.3 and Algorithm 1: every particle walks the tree without a
 *     stack (descend on overlap, follow the rope otherwise), once per
 *     periodic image whose search sphere touches the root box, testing a
 *     sphere against each box with the nearest-point rule of eq. (2).
 *
 * This library returns exact lists: where the paper accepts every particle
 * whose leaf box the sphere overlaps, each candidate is decided here by the
 * fp64 minimum-image distance, so the result is exactly
 *
 *   S_i = { j != i : d_ij <= rcut[t_i][t_j] + skin }       (rcut > 0 only)
 *
 * with d_ij evaluated in fp64 from the fp32 coordinates as
 *   dx_d = (x_j,d - x_i,d) - L_d * round((x_j,d - x_i,d) / L_d),
 *   d^2  = (dx_0*dx_0 + dx_1*dx_1) + dx_2*dx_2   (no fused multiply-add)
 * and compared with (rcut + skin)^2 computed in fp64.
 *
 * Conventions for every call:
 *   - Pointers named d_* are device pointers (hipMalloc or torch CUDA
 *     tensors).  Everything else is host memory.
 *   - qbvh_stream_t is a hipStream_t; NULL means the default stream.  All
 *     calls enqueue work on the stream and return without waiting, unless
 *     stated otherwise.  Inputs must stay valid until that work completes.
 *   - Return value: QBVH_OK (0) or a negative QBVH_E* code; no exception or
 *     abort crosses this interface.  qbvh_strerror() names the code.
 *   - One handle may be used by one stream at a time; concurrent calls on
 *     different handles are independent.
 */
#ifndef QBVH_H
#define QBVH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__) || defined(__clang__)
#define QBVH_API __attribute__((visibility("default")))
#else
#define QBVH_API
#endif

typedef struct qbvh qbvh_t;   /* opaque: a built tree plus its device workspace */
typedef void *qbvh_stream_t;  /* hipStream_t */

enum {
    QBVH_OK = 0,
    QBVH_EINVAL = -1, /* bad argument: NULL pointer, n outside 0..2^27-1, ntypes outside 1..4,
                         box edge <= 0 or not finite, skin < 0, rcut not symmetric,
                         max_nbr < 0, unsupported option value, or (with
                         validate) a coordinate outside [0, L) or a type outside
                         [0, ntypes) */
    QBVH_EGEOM = -2,  /* 2 * max(rcut + skin) >= min box edge: the minimum image
                         would not be unique */
    QBVH_ENOMEM = -3, /* device allocation failed */
    QBVH_EHIP = -4,   /* a HIP runtime call failed; qbvh_last_hip_error() has it */
    QBVH_EAGAIN = -5, /* server admission: the request does not fit right now */
    QBVH_ENOTSUP = -6, /* valid request the library does not support */
    QBVH_ENOSPACE = -7 /* nlist_build_noalloc: n needs more than QBVH_NOALLOC_BYTES of workspace */
};

#define QBVH_MAX_TYPES 4

/* Build options.  A NULL pointer, or a zero field, selects the default. */
typedef struct {
    int32_t leaf_size;  /* particles per leaf run: a subtree with at most this many
                           particles is not split further and its particles are
                           tested one by one (1..16, default 16; 1 gives one particle
                           per leaf as in the paper) */
    int32_t qbits;      /* grid bits per axis for the quantized bounds (8..16,
                           default 16; the paper's layout uses 10) */
    int32_t block_size; /* traversal workgroup size: 64, 128, 192 or 256
                           (default 64) */
    int32_t validate;   /* 1: check every coordinate and type on the device and
                           wait for the result (the call then synchronizes the
                           stream); 0 (default): inputs are trusted */
    float collapse_radius; /* subtree collapse (Section 2.3, last paragraph).  0 (default):
                           every subtree of at most leaf_size particles is one leaf run.
                           > 0: the tree is built with one particle per leaf and a subtree
                           of at most leaf_size particles is collapsed into a run only when
                           a cost estimate for search spheres of this radius (the expected
                           list radius) says so: testing its particles (cost 1 each) must
                           cost no more than testing its children's boxes (a record, cost
                           4) plus the expected cost of the children, the chance that a
                           sphere meets a box being taken proportional to the box's volume
                           grown by the radius.  Must be finite and >= 0. */
    int32_t queries_per_wave; /* queries that share one wavefront's walk: 1, 2, 4, 8, 16, 32
                           or 64; 0 (default) chooses from the system size (64 for large
                           systems, fewer for small ones) */
} qbvh_opts_t;

/*
 * qbvh_build -- build the quantized BVH of every particle type (Section 2.1,
 * Section 2.2, Fig. 3b).
 *
 *   tree    in/out.  *tree == NULL: a new handle is allocated.  *tree != NULL:
 *           a handle from an earlier call, rebuilt in place (its workspace is
 *           kept when large enough, otherwise reallocated after waiting for
 *           its pending work).  Release with qbvh_free().
 *   d_pos   device float [n][3], x y z of particle i at 3i..3i+2, every
 *           coordinate in [0, box[d]).
 *   d_type  device int32 [n] with values in [0, ntypes), or NULL when ntypes == 1.
 *   n       number of particles, 0 .. 2^27 - 1 (0: an empty tree, no work).
 *   ntypes  1..4; one tree is built per type (types with no particles give
 *           empty trees).
 *   box     host float [3]: orthorhombic periodic box edges, all > 0.
 *   opts    NULL or options (see qbvh_opts_t).
 *
 * The library owns the handle and its device memory; d_pos and d_type are
 * only read, by work enqueued on the stream.
 */
QBVH_API int qbvh_build(qbvh_t **tree, const float *d_pos, const int32_t *d_type, int32_t n,
               int32_t ntypes, const float box[3], const qbvh_opts_t *opts,
               qbvh_stream_t stream);

/*
 * qbvh_build_f64 -- the same build for fp64 particle data (the paper's fp64
 * case: Section 2.2, where fp32 bounds that contain the fp64 data keep the
 * tree small, and Figs. 4-7).
 *
 *   d_pos   device double [n][3], every coordinate in [0, box[d]).
 *   box     host double [3]: box edges, all > 0 and finite.
 *   (tree, d_type, n, ntypes, opts as qbvh_build.)
 *
 * The tree is built and walked on the positions rounded to fp32; the fp64
 * positions are kept in sorted order, and every pair whose fp32 distance is
 * within the rounding band of the cutoff is decided with them.  nlist_build
 * on such a tree returns the exact list of the fp64 data (the definition at
 * the top with dx computed from the fp64 coordinates and the fp64 box).
 * Paper-mode lists (nlist_build_ex with QBVH_LIST_PAPER) return QBVH_ENOTSUP
 * for it.  d_pos must stay valid until the build's work on the stream is done.
 * Errors as qbvh_build; validate = 1 checks the fp64 coordinates.
 */
QBVH_API int qbvh_build_f64(qbvh_t **tree, const double *d_pos, const int32_t *d_type, int32_t n,
                   int32_t ntypes, const double box[3], const qbvh_opts_t *opts,
                   qbvh_stream_t stream);

/*
 * nlist_build -- traverse the tree once per particle (Algorithm 1, eq. (2),
 * Section 2.3) and write the exact neighbor list defined at the top.
 *
 *   rcut      host float [ntypes][ntypes], row-major, symmetric; a pair of
 *             types with rcut <= 0 is never listed.
 *   skin      list buffer added to every cutoff (>= 0).
 *   max_nbr   row capacity (>= 0; 0 = counts only, d_nbr may then be NULL).
 *   d_nbr     device int32 [n][max_nbr] (caller-owned).  Row i lists the
 *             ORIGINAL indices of the neighbors of input particle i in its first
 *             min(count_i, max_nbr) slots; the remaining slots are untouched.
 *             Order within a row is unspecified but identical from run to run.
 *             When max_nbr is a multiple of 4 and d_nbr is 16-byte aligned, rows
 *             are written with 16-byte stores.
 *   d_count   device int32 [n]: the true |S_i|, also when it exceeds max_nbr.
 *   d_overflow device int32 [1]: set to 1 if some count exceeds max_nbr, else 0.
 *             Overflow is not an error; the caller reads the flag after syncing.
 *
 * The list is full and symmetric: j is in row i exactly when i is in row j.
 */
QBVH_API int nlist_build(const qbvh_t *tree, const float *rcut, float skin, int32_t max_nbr,
                int32_t *d_nbr, int32_t *d_count, int32_t *d_overflow, qbvh_stream_t stream);

/* List semantics of nlist_build_ex. */
enum {
    QBVH_LIST_EXACT = 0, /* the exact list defined at the top (what nlist_build writes) */
    QBVH_LIST_PAPER = 1  /* the paper's lists (Section 2.3): j is listed for i when i's
                            sphere (radius R = rcut[t_i][t_j] + skin, any periodic image)
                            overlaps j's cell box -- j's position snapped outward to the
                            grid of its type's tree, the leaf box of a one-particle leaf --
                            with no distance check.  The grid is the paper's (Section 2.2):
                            the tree's root-node box split into 2^qbits - 1 bins along
                            each axis, of width h_d = extent_d / (2^qbits - 1).  A superset
                            of the exact list; the extra entries are the paper's false
                            positives (about rho (hx hy hz + 2 R (hx hy + hy hz + hz hx)
                            + pi R^2 (hx + hy + hz)) per particle).  The test uses the
                            radius R (1 + 2^-20) + 0.02 max_d h_d, which covers its
                            rounding; the relation is not symmetric. */
};

/*
 * nlist_build_ex -- nlist_build with a choice of list semantics (`mode`, one
 * of QBVH_LIST_*; anything else is QBVH_EINVAL).  Paper mode first writes
 * every particle's cell box into the tree's workspace (stream-ordered).
 * Arguments, layouts and outputs otherwise as nlist_build.
 */
QBVH_API int nlist_build_ex(const qbvh_t *tree, const float *rcut, float skin, int32_t max_nbr, int32_t mode,
                   int32_t *d_nbr, int32_t *d_count, int32_t *d_overflow, qbvh_stream_t stream);

/* One independent system of a batch. */
typedef struct {
    const float *d_pos;    /* device float [n][3] */
    const int32_t *d_type; /* device int32 [n] or NULL when ntypes == 1 */
    int32_t n;
    int32_t ntypes;
    float box[3];
    const float *rcut;     /* host float [ntypes][ntypes] */
    float skin;
    int32_t max_nbr;
    int32_t *d_nbr;        /* device int32 [n][max_nbr] */
    int32_t *d_count;      /* device int32 [n] */
    int32_t *d_overflow;   /* device int32 [1] */
} qbvh_system_t;

typedef struct {
    int32_t leaf_size;  /* as qbvh_opts_t; 0 = let the autotuner choose */
    int32_t qbits;      /* as qbvh_opts_t; 0 = let the autotuner choose */
    int32_t block_size; /* as qbvh_opts_t; 0 = let the autotuner choose */
    int32_t eager;      /* 0 (default): capture the launch sequence of each batch
                           shape and configuration once in a hipGraph and replay
                           it; 1: launch the kernels directly on every call */
} qbvh_batch_opts_t;

/*
 * nlist_build_many -- build the trees of many independent systems and write
 * their exact lists in one launch sequence (Section 2.1 to Section 2.3 per
 * system; the paper builds one system at a time, here every kernel covers
 * all systems at once).
 *
 *   nsys    number of systems (0: no work).
 *   sys     host array [nsys]; each entry as for qbvh_build + nlist_build
 *           (d_pos/d_type/n/ntypes/box as qbvh_build, rcut/skin/max_nbr and
 *           the outputs as nlist_build).  Inputs are trusted (no device
 *           validation); the sum of n must stay below 2^27.
 *   opts    NULL or options; a zero field is chosen by the autotuner.
 *
 * Each system's outputs equal those of qbvh_build + nlist_build on that
 * system alone: the same neighbor sets and identical counts (row order may
 * differ).  The library keeps, per stream and device, a batch context: a
 * workspace that grows as needed (growing waits for the stream) and, per
 * batch shape (the list of n and ntypes, and whether all rows take 16-byte
 * stores), the autotuner state and the captured graphs.  While tuning, the
 * calls of one shape cycle through the candidate configurations, each timed
 * twice with events, then the fastest is kept for that shape.  Pointers,
 * boxes and cutoffs may change between calls of one shape; they live in a
 * device table uploaded before the launch when it changed.  Calls on one
 * stream are serialized by the library; overlapping calls on different
 * streams use different contexts.
 */
QBVH_API int nlist_build_many(int32_t nsys, const qbvh_system_t *sys, const qbvh_batch_opts_t *opts,
                     qbvh_stream_t stream);

/* Autotuner state of the last batch shape used on a stream. */
typedef struct {
    int32_t tuned;           /* 1 once the configuration is frozen */
    int32_t leaf_size, qbits, block_size;  /* the chosen configuration (first candidate while tuning) */
    int32_t candidates;      /* configurations in the search */
    int32_t graphs_captured; /* graphs captured for this shape so far */
    int64_t calls;           /* calls of this shape */
    float best_ms;           /* fastest measured call of the chosen configuration (0 if none) */
} qbvh_batch_stats_t;

QBVH_API int nlist_batch_stats(qbvh_stream_t stream, qbvh_batch_stats_t *out);

/* Free the batch context of a stream on the current device (waits for the
 * stream first).  Unknown streams are ignored. */
QBVH_API void nlist_batch_release(qbvh_stream_t stream);

/* ---------------------------------------------------------------- serving */

/*
 * A server accepts rebuild requests from many concurrent simulations and
 * serves them with continuous batching: a worker thread keeps up to
 * `max_inflight` batches on the device (one stream each); whenever a stream
 * is free it takes every queued request that is admissible right now and
 * launches them together as one nlist_build_many call, so requests that
 * arrive while others run are admitted as soon as a stream and memory free
 * up, and their work overlaps on the device.
 *
 * Sessions.  Every sim_id owns a session holding result buffers (list,
 * counts and overflow flag) in device memory.  The buffer of the sim's last
 * completed request is its published result, resident until the sim's next
 * request replaces it or the session is evicted.  (The tree is rebuilt on
 * every request, as the method rebuilds it at every list update, so it lives
 * only in the batch workspace.)  Requests of one sim run one at a time, in
 * submission order.
 *
 * Results are read under a lease: qbvh_server_result hands out the published
 * buffer and leases it; a leased buffer is neither written nor freed until
 * qbvh_server_release returns the lease.  A client may submit the sim's next
 * request before releasing: it runs into another buffer.
 *
 * Admission by footprint.  A request needs one result buffer
 * (n * max_nbr * 4 + n * 4 + 4 bytes, each part rounded up to 256) that no
 * lease holds, plus its share of its stream's batch workspace (about
 * qbvh_workspace_bytes of the batch's particles).  In order of preference it
 * writes: a spare buffer of its session that is large enough; a new buffer,
 * if one fits after freeing spare buffers; its published buffer, if no lease
 * holds it (the sim has no published result while the request runs); a new
 * buffer after evicting whole idle sessions that hold no lease, least
 * recently used first (an evicted sim's result is gone: qbvh_server_result
 * then returns QBVH_EINVAL).  It is admitted when the bytes of all result
 * buffers and of every stream's workspace, with its own, fit in
 * `budget_bytes`.  A request that could never fit is refused at submission
 * with QBVH_EAGAIN; otherwise it waits in FIFO order (a request that does not
 * fit yet does not block smaller ones behind it).  When nothing is running
 * and no queued request fits even with the streams' workspaces released, the
 * budget is held by leased buffers: those requests complete with
 * QBVH_EAGAIN.  So every submitted request completes, with its results or
 * with an error.
 */
typedef struct qbvh_server qbvh_server_t;

typedef struct {
    size_t budget_bytes;      /* device bytes for sessions plus batch workspaces (> 0) */
    int32_t max_inflight;     /* batches on the device at once, 1..8 (0: 2) */
    int32_t max_batch;        /* requests per batch, >= 1 (0: 64) */
    qbvh_batch_opts_t batch;  /* options of the batched launches; zero fields take
                                 leaf 16, 16 bits, 128 work-items; graphs are not used
                                 (every batch has a new composition) */
} qbvh_server_opts_t;

typedef struct {
    int32_t sim_id;           /* session key (>= 0) */
    const float *d_pos;       /* device float [n][3]; read on the server's own streams, so it
                                 must already hold its values when submitted (the work that
                                 wrote it has completed) and stay valid until the request
                                 completes */
    const int32_t *d_type;    /* device int32 [n] or NULL when ntypes == 1 (same lifetime) */
    int32_t n, ntypes;
    float box[3];
    const float *rcut;        /* host float [ntypes][ntypes]; copied at submission */
    float skin;
    int32_t max_nbr;          /* >= 1 */
} qbvh_request_t;

typedef struct {
    int64_t submitted, completed, batches, refused;
    double p50_ms, p99_ms, mean_ms;  /* latency: submission to completion seen by the worker */
    double requests_per_s;           /* completed requests / (last completion - first submission) */
    double particles_per_s;          /* particles of completed requests over the same span */
    double mean_batch;               /* requests per batch */
    size_t bytes_resident;           /* session buffers held now */
    size_t bytes_peak;               /* peak of sessions + in-flight workspaces */
} qbvh_server_stats_t;

/* Create a server on the current device.  Returns QBVH_EINVAL for bad options. */
QBVH_API int qbvh_server_create(qbvh_server_t **srv, const qbvh_server_opts_t *opts);

/* Queue a request; *ticket receives its id (> 0).  Arguments are checked as
 * for qbvh_build + nlist_build (QBVH_EINVAL / QBVH_EGEOM); QBVH_EAGAIN if the
 * request can never fit the budget.  Never blocks on the device. */
QBVH_API int qbvh_server_submit(qbvh_server_t *srv, const qbvh_request_t *req, int64_t *ticket);

/* *done = 1 once the request has finished (its results, if any, are on the
 * device), else 0; a finished request's return is its status (QBVH_OK or the
 * error it failed with).  QBVH_EINVAL for an unknown ticket.  A ticket is
 * forgotten once poll or wait has reported it finished. */
QBVH_API int qbvh_server_poll(qbvh_server_t *srv, int64_t ticket, int32_t *done);

/* Block until the request finishes; returns its status (one waiter per ticket). */
QBVH_API int qbvh_server_wait(qbvh_server_t *srv, int64_t ticket);

/* Lease the published result of a sim: d_nbr [n][max_nbr], d_count [n],
 * d_overflow [1], as nlist_build writes them, for its last completed request
 * (any output pointer may be NULL).  The buffers stay valid and unchanged
 * until the lease is returned with qbvh_server_release(srv, sim_id, *d_nbr);
 * every successful call takes one lease.  QBVH_EINVAL for an unknown sim, one
 * with nothing completed, or one whose session was evicted. */
QBVH_API int qbvh_server_result(qbvh_server_t *srv, int32_t sim_id, const int32_t **d_nbr, const int32_t **d_count,
                       const int32_t **d_overflow, int32_t *n, int32_t *max_nbr);

/* Return one lease of a sim's result buffer, named by the d_nbr pointer that
 * qbvh_server_result gave.  QBVH_EINVAL if no such lease is held.  Device
 * work that reads the buffers must be ordered before the release by the
 * caller (e.g. synchronize the stream that reads them). */
QBVH_API int qbvh_server_release(qbvh_server_t *srv, int32_t sim_id, const int32_t *d_nbr);

QBVH_API int qbvh_server_stats(qbvh_server_t *srv, qbvh_server_stats_t *stats);

/* Finish every queued and running request (each completes or fails as
 * described above), then free the server and every session; leases end.
 * No other call on the server may run concurrently with it. */
QBVH_API void qbvh_server_destroy(qbvh_server_t *srv);

/* ------------------------------------------------------- without allocation */

/* Size of the fixed workspace of nlist_build_noalloc (160 MiB on each GPU the
 * library runs on; about 153.5 bytes per particle, so n up to about 1.09
 * million: qbvh_workspace_bytes(n, ...) <= QBVH_NOALLOC_BYTES). */
#define QBVH_NOALLOC_BYTES ((size_t)160 << 20)

/*
 * nlist_build_noalloc -- qbvh_build followed by nlist_build in one call that
 * allocates no memory, for callers that cannot allocate: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 *
 * The tree is built into a fixed workspace of QBVH_NOALLOC_BYTES that the
 * library holds in its code object, one per GPU, from its first use on that
 * GPU until the process ends; the call makes no hipMalloc, hipFree or other
 * allocating call.  Because the next call overwrites that workspace, the tree
 * is not kept: build and list are one call.
 *
 *   d_pos, d_type, n, ntypes, box, opts   as qbvh_build (fp32 data)
 *   rcut, skin, max_nbr, d_nbr, d_count, d_overflow   as nlist_build
 *
 * Outputs are those of qbvh_build + nlist_build with the same arguments,
 * entry for entry.  Errors as those two calls, plus QBVH_ENOSPACE when n needs
 * more workspace than QBVH_NOALLOC_BYTES (nothing is launched then).
 * opts->validate = 1 synchronizes the stream, as in qbvh_build.
 *
 * Every call on one GPU uses that GPU's one workspace: calls ordered on one
 * stream are safe, but calls whose work overlaps on one GPU (different
 * streams or threads without ordering between them) race and give wrong
 * lists.  The first call on a GPU looks up the workspace's device address
 * (a runtime query, no allocation).
 */
QBVH_API int nlist_build_noalloc(const float *d_pos, const int32_t *d_type, int32_t n, int32_t ntypes,
                    const float box[3], const qbvh_opts_t *opts, const float *rcut, float skin,
                    int32_t max_nbr, int32_t *d_nbr, int32_t *d_count, int32_t *d_overflow,
                    qbvh_stream_t stream);

/* Release a handle (waits for its pending work).  NULL is ignored. */
QBVH_API void qbvh_free(qbvh_t *tree);

/* Static description of a return code. */
QBVH_API const char *qbvh_strerror(int code);

/* The hipError_t value of the most recent QBVH_EHIP on this thread. */
QBVH_API int qbvh_last_hip_error(void);

/* Device bytes qbvh_build allocates for n particles (for admission control). */
QBVH_API size_t qbvh_workspace_bytes(int32_t n, int32_t ntypes, const qbvh_opts_t *opts);

/* ---------------------------------------------------------------- inspection */

/* Host-side summary of a built tree.  Synchronizes the handle's last stream. */
typedef struct {
    int32_t n, ntypes, nrecords, leaf_size, qbits;
    int32_t tree_start[QBVH_MAX_TYPES]; /* first sorted index of each type */
    int32_t tree_count[QBVH_MAX_TYPES]; /* particles of each type */
    int32_t tree_root[QBVH_MAX_TYPES];  /* root record of each tree, or (trees of at most
                                           leaf_size particles) the run reference below */
    int32_t tree_end[QBVH_MAX_TYPES];   /* one past each tree's last record */
    float root_lo[QBVH_MAX_TYPES][3];   /* root-node box of each tree */
    float root_hi[QBVH_MAX_TYPES][3];
    double h[QBVH_MAX_TYPES];           /* grid spacing of each tree */
} qbvh_info_t;

QBVH_API int qbvh_info(const qbvh_t *tree, qbvh_info_t *info);

/* Intermediate arrays of the last build, copied device-to-device into a
 * caller buffer of at least the stated size (stream-ordered). */
enum {
    QBVH_EXPORT_KEYS = 1,    /* uint32 [n]  sorted keys: (type << 30) | Morton code */
    QBVH_EXPORT_PERM = 2,    /* uint32 [n]  original index of each sorted position */
    QBVH_EXPORT_SORTED = 3,  /* float4 [n]  sorted x, y, z and w = bits of ~original index */
    QBVH_EXPORT_LEFT = 4,    /* int32 [n]   left child of internal node i (leaf k as ~k) */
    QBVH_EXPORT_RIGHT = 5,   /* int32 [n]   right child of internal node i */
    QBVH_EXPORT_RANGE_F = 6, /* int32 [n]   first sorted position below internal node i */
    QBVH_EXPORT_RANGE_L = 7, /* int32 [n]   last sorted position below internal node i */
    QBVH_EXPORT_PARENT = 8,  /* int32 [n]   parent of internal node i (-1 at a root) */
    QBVH_EXPORT_LEAF_PARENT = 9, /* int32 [n] parent of leaf k (-1 for a one-particle tree) */
    QBVH_EXPORT_BOX_LO = 10, /* float4 [n]  lower box corner of internal node i */
    QBVH_EXPORT_BOX_HI = 11, /* float4 [n]  upper box corner of internal node i */
    QBVH_EXPORT_RECORDS = 12, /* uint32 [nrecords][8] two-wide quantized records:
                                 words 0-2 left child box, 3-5 right child box
                                 (q_lo | q_hi << 16 per axis), 6 left child,
                                 7 right child: record index, or a particle run
                                 ~((first << 4) | (count - 1)) */
    QBVH_EXPORT_ROPES = 13    /* int32 [nrecords] record that follows each record's subtree */
};
/* Internal node ids are sorted positions: the tree of the type occupying
 * sorted positions [s, e) has internal nodes s .. e-2; entries for other ids
 * are unspecified. */
QBVH_API int qbvh_export(const qbvh_t *tree, int32_t what, void *d_dst, size_t dst_bytes,
                qbvh_stream_t stream);

/*
 * nlist_build_grid -- the same exact list (one particle type) by the grid
 * method the paper compares its tree with (Section 1, Section 3 and
 * Section 4: particles sorted into a uniform grid of cells at least as wide
 * as the list radius; each particle tests the particles of the 27 cells
 * around its own, with n cooperating lanes per particle).  It exists to
 * measure the tree against a grid on the same GPU.
 *
 *   grid    in/out.  *grid == NULL: a new handle is allocated (release with
 *           qgrid_free); otherwise its device workspace is reused, and
 *           reallocated after waiting for its pending work when too small.
 *   d_pos, n, box   as qbvh_build (n >= 0; coordinates in [0, box[d])).
 *   rcut, skin      list radius rcut + skin (rcut > 0, skin >= 0).
 *   lanes   lanes per particle n: 1, 2, 4, 8, 16 or 32 (0: 4).  The n lanes
 *           take a cell's candidates n at a time and combine their accepted
 *           ones within the group; the paper picks the fastest n per system.
 *   max_nbr, d_nbr, d_count, d_overflow   as nlist_build (rows hold original
 *           indices in the order the cells and candidates are scanned, the
 *           same from run to run for a given lanes).
 *
 * Cells per axis: floor(L_d / r_list), at most 1024.  Returns QBVH_EGEOM when
 * 2 r_list >= min L_d, QBVH_ENOTSUP when an axis would hold fewer than 3
 * cells, QBVH_EINVAL for a lanes value not listed.  Asynchronous on the
 * stream; d_pos must stay valid until the work is done.  Inputs are trusted
 * (no device validation).
 */
typedef struct qgrid qgrid_t;
QBVH_API int nlist_build_grid(qgrid_t **grid, const float *d_pos, int32_t n, const float box[3], float rcut,
                     float skin, int32_t lanes, int32_t max_nbr, int32_t *d_nbr, int32_t *d_count,
                     int32_t *d_overflow, qbvh_stream_t stream);
QBVH_API void qgrid_free(qgrid_t *grid);

#ifdef __cplusplus
}
#endif

#endif /* QBVH_H */

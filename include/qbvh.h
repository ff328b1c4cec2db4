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
 *     fit bottom-up, giving N - 1 internal nodes with two children each;
 *   - Section 2.2: node bounds are snapped outward to an integer grid over
 *     the root-node box and packed, with a skip rope, into 16-byte nodes;
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
    QBVH_EINVAL = -1, /* bad argument: NULL pointer, n outside 0..2^28-1, ntypes outside 1..4,
                         box edge <= 0 or not finite, skin < 0, rcut not symmetric,
                         max_nbr < 0, unsupported option value, or (with
                         validate) a coordinate outside [0, L) or a type outside
                         [0, ntypes) */
    QBVH_EGEOM = -2,  /* 2 * max(rcut + skin) >= min box edge: the minimum image
                         would not be unique */
    QBVH_ENOMEM = -3, /* device allocation failed */
    QBVH_EHIP = -4,   /* a HIP runtime call failed; qbvh_last_hip_error() has it */
    QBVH_EAGAIN = -5, /* server admission: the request does not fit right now */
    QBVH_ENOTSUP = -6 /* valid request this build does not support */
};

#define QBVH_MAX_TYPES 4

/* Build options.  A NULL pointer, or a zero field, selects the default. */
typedef struct {
    int32_t leaf_size;  /* particles per leaf run: a subtree with at most this many
                           particles is not split further and its particles are
                           tested one by one (1..8, default 1 = one particle per
                           leaf as in the paper) */
    int32_t qbits;      /* grid bits per axis for the quantized bounds (8..16,
                           default 16; the paper's layout uses 10) */
    int32_t block_size; /* traversal workgroup size: 64, 128, 192 or 256
                           (default 256) */
    int32_t validate;   /* 1: check every coordinate and type on the device and
                           wait for the result (the call then synchronizes the
                           stream); 0 (default): inputs are trusted */
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
 *   n       number of particles, 0 .. 2^28 - 1 (0: an empty tree, no work).
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
    int32_t use_graph;  /* 1: capture the launch sequence in a hipGraph and replay
                           it while the batch shape is unchanged (default 1) */
} qbvh_batch_opts_t;

/*
 * nlist_build_many -- build and traverse many independent systems in one
 * launch sequence (every build phase covers all systems at once).  Each
 * system's outputs equal those of qbvh_build + nlist_build on that system
 * alone (same sets, same counts).  The library keeps a batch workspace that
 * grows as needed.
 */
QBVH_API int nlist_build_many(int32_t nsys, const qbvh_system_t *sys, const qbvh_batch_opts_t *opts,
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
                                 ~((first << 3) | (count - 1)) */
    QBVH_EXPORT_ROPES = 13    /* int32 [nrecords] record that follows each record's subtree */
};
/* Internal node ids are sorted positions: the tree of the type occupying
 * sorted positions [s, e) has internal nodes s .. e-2; entries for other ids
 * are unspecified. */
QBVH_API int qbvh_export(const qbvh_t *tree, int32_t what, void *d_dst, size_t dst_bytes,
                qbvh_stream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* QBVH_H */

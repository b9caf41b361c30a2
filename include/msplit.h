/*
 * msplit.h -- C ABI of libmsplit, an MI355X (gfx950) splitter for the
 * Mandelbrot polynomials of Mihalache & Vigneron, "How to split a
 * tera-polynomial" (arXiv 2402.06083):
 *
 *   p_n(c)     = f_c^n(0),  f_c(z) = z^2 + c,  deg p_n = 2^(n-1)
 *                (Section 1, eq. def:hyp_poly; roots = hyperbolic centres)
 *   q_{l,n}(c) = p_{l+n}(c) - p_l(c),  deg = 2^(l+n-1)
 *                (Section 1, eq. def:mis_poly; roots include Mis(l,n))
 *
 * A splitting call returns the list of all roots (Section 3: a splitting
 * algorithm provides the list of all the roots of P), found by the level-line
 * method of Section 4: starting points on the discrete level line
 * L_{lambda_0, 4d}(P) (Thm practicalFTA, Prop. computeLevelLine, Algorithm
 * S_par), a capped Newton descent from each of them, collection in the nset
 * sense (Section 6.1) and, on request, the disk-arithmetic certificate of
 * Thm proofRoots / Thm certif (Section 5, Section 6.2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Array pointers inside msplit_roots and the workspace are HIP DEVICE
 *   pointers owned by the caller.  Scalars (counts, stats) are HOST pointers.
 *   The library never allocates or frees device memory; it uses the
 *   workspace only, whose size msplit_workspace_size() reports (except
 *   msplit_hyperbolic_static, which runs in a static device array of the
 *   library instead).
 * - stream is a hipStream_t (NULL = the null stream).  Kernels are enqueued
 *   on it; every entry point synchronises that stream before returning
 *   because it reports counts on the host.  Calls on distinct streams with
 *   distinct workspaces may run concurrently; calls sharing a workspace must
 *   not overlap.
 * - Roots are returned in the closed upper half plane (Section 6.1: only
 *   Im >= 0 is stored; p_n and q_{l,n} have integer coefficients): a real
 *   root appears once with im == 0 exactly, a non-real root stands for
 *   itself and its conjugate (MSPLIT_F_CONJUGATES writes both).  Order: increasing real part, to 2^-46 (roots
 *   whose real parts are closer than that come in start order).  Where FP64 cannot separate the roots (next to c = -2) a root is
 *   a double-double value re + re_lo, im + im_lo (flag MSPLIT_R_DD); give
 *   re_lo and im_lo to receive the low parts (otherwise such roots are
 *   returned to FP64 only).
 * - Return value: MSPLIT_OK (0) or a negative msplit_status.  No C++
 *   exception crosses the ABI.
 */
#ifndef MSPLIT_H
#define MSPLIT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status */
enum msplit_status {
    MSPLIT_OK = 0,
    MSPLIT_E_ARG = -1,        /* bad (l, n), null pointer, bad option */
    MSPLIT_E_CAPACITY = -2,   /* output capacity too small; *count holds the need */
    MSPLIT_E_WORKSPACE = -3,  /* workspace smaller than msplit_workspace_size() */
    MSPLIT_E_DEVICE = -4,     /* a HIP call failed (stats->hip_error holds it) */
    MSPLIT_E_INCOMPLETE = -5, /* fewer roots than the exact count (stats->missing) */
    MSPLIT_E_PRECISION = -6,  /* the requested precision cannot separate the roots */
    MSPLIT_E_UNSUPPORTED = -7 /* valid request this build does not implement */
};

/* --------------------------------------------------------------- precision */
enum msplit_precision {
    MSPLIT_FP64 = 0,  /* walk and descent in FP64 */
    MSPLIT_MIXED = 1, /* descent starts in FP32, FP64 refinement */
    MSPLIT_DD = 2     /* every descent in double-double from its starting point (Section 6.4.3:
                         the high-precision tier for a whole job); every root is a double-double
                         value (MSPLIT_R_DD: msplit_roots.re_lo and im_lo are required, else
                         MSPLIT_E_ARG), identified, classified and certified in double-double */
};

/* ------------------------------------------------------------------- flags */
enum msplit_flags {
    MSPLIT_F_CERTIFY = 1u, /* run the disk-arithmetic certificate (Thm proofRoots) */
    MSPLIT_F_NO_LABEL = 2u, /* skip period / type classification */
    MSPLIT_F_BASIN = 4u,    /* with MSPLIT_F_CERTIFY and msplit_roots.basin: prove a disk of
                               Newton convergence around every certified root (Thm proofContract) */
    MSPLIT_F_SIMPLE = 8u,   /* Misiurewicz types: find Mis(l,n) among the roots of the simplified
                               polynomial s_{l,n} = p_{l+n-1} + p_{l-1} = q_{l,n} / q_{l-1,n}
                               (eq. polySimple: simple roots, half the degree of q_{l,n}); the
                               certificate still applies Thm proofRoots to q_{l,n} */
    MSPLIT_F_CONJUGATES = 16u /* write all the roots of P, not the upper half plane only: each
                                 non-real root preceded by its conjugate (order: real part, then
                                 imaginary part); the conjugate carries the same label, radius and
                                 basin (P has real coefficients).  The capacity must hold every root
                                 (2^(n-1) for p_n), else MSPLIT_E_CAPACITY.  Not with
                                 msplit_split_streamed (MSPLIT_E_UNSUPPORTED) */
};

/* per-root flag bits written to msplit_roots.flags */
enum msplit_root_flags {
    MSPLIT_R_REAL = 1u,      /* im == 0: the root is real (proven when certified) */
    MSPLIT_R_CERTIFIED = 2u, /* D(root, radius) holds exactly one root of P */
    MSPLIT_R_LABEL = 4u,     /* the period / type label is proven on that disk */
    MSPLIT_R_DD = 8u,        /* double-double root: the value is re + re_lo, im + im_lo (roots
                                next to -2 that FP64 cannot separate); certified in double-double */
    MSPLIT_R_BASIN = 16u     /* D(root, basin) lies in the Newton basin of the root (Thm
                                proofContract; root = re + re_lo, im + im_lo for a DD root) */
};

/* Device workspace, in bytes, that msplit_certify needs (counters and one
 * type descriptor; independent of the number of candidates). */
#define MSPLIT_CERTIFY_WORKSPACE 16384u

/* Options.  Zero in any field selects the default shown. */
typedef struct msplit_options {
    uint32_t struct_size;     /* sizeof(msplit_options) */
    int32_t precision;        /* msplit_precision, default MSPLIT_FP64 */
    double level;             /* lambda_0: 5 for p_n, 100 for q_{l,n} (Section 4.2) */
    uint32_t points_per_turn; /* M, level-line points per turn: 8 (Section 6.3.1) */
    uint32_t seg_points;      /* fine level-line points per segment (a power of two,
                                 at least 2; each segment is walked from both of
                                 its seeds to its middle point): auto */
    uint32_t min_cap;         /* Newton cap floor: 20 (Algorithm S_par) */
    double cap_factor;        /* I_N of the cap max{20, I_N log d}: 1 (p), 2.6 (q) */
    uint32_t block_size;      /* threads per block: 256 */
    uint32_t flags;           /* msplit_flags */
    double fp32_switch;       /* MIXED: relative step at which a lane leaves FP32: 2^-14 */
} msplit_options;

/* Output arrays (device pointers, each of `capacity` elements). */
typedef struct msplit_roots {
    double *re, *im;       /* root centres */
    double *re_lo, *im_lo; /* nullable: low parts of a double-double root */
    int32_t *period;       /* nullable: p_n: exact period k | n; q_{l,n}: n */
    int32_t *preperiod;    /* nullable: q_{l,n}: l; p_n: 0 */
    uint8_t *flags;        /* nullable: msplit_root_flags */
    double *radius;        /* nullable: certificate radius (0 if not certified) */
    uint64_t capacity;
    double *basin;         /* nullable: Newton-basin radius eps_N (0 if not proven); written
                              with MSPLIT_F_BASIN (msplit_certify: whenever non-null) */
} msplit_roots;

/* Statistics (host). */
typedef struct msplit_stats {
    uint64_t starts;        /* level-line starting points (closed upper half plane) */
    uint64_t converged;     /* descents that converged */
    uint64_t diverged;      /* descents discarded as divergent */
    uint64_t timeouts;      /* descents that hit the cap */
    uint64_t unique;        /* roots after collection */
    uint64_t n_real;        /* real roots among them */
    uint64_t total;         /* n_real + 2 (unique - n_real): roots counted in C */
    uint64_t expected;      /* exact count: 2^(n-1) for p_n, |Mis(l,n)| for q */
    uint64_t missing;       /* expected - total when positive */
    uint64_t phase_fail;    /* level-line segments whose FP64 walk missed the next seed (their
                               starts are then lifted again in double-double, one by one),
                               plus seed and double-double lifts that did not converge */
    uint64_t certified;     /* roots with MSPLIT_R_CERTIFIED */
    uint64_t label_proven;  /* roots with MSPLIT_R_LABEL */
    uint64_t overlaps;      /* certified disks that are not quarter-separated */
    uint64_t steps_lift;    /* polynomial evaluations in the seed lift */
    uint64_t steps_walk;    /* ... in the level-line walk */
    uint64_t steps_desc;    /* ... in the descents */
    uint64_t steps_fp32;    /* ... of which in FP32 (MIXED) */
    uint64_t sorted;        /* converged starts left after the local identification of
                               consecutive starts: the entries of the global sort */
    uint64_t discarded;     /* identified roots of a lower type dropped by the
                               classification (q_{l,n}: Hyp(k), Mis(j,k) with j < l or
                               k < n; zero for p_n) */
    uint64_t dd_routed;     /* descents redone in double-double next to -2 */
    uint64_t steps_dd;      /* polynomial evaluations of those descents */
    double min_sep;         /* least distance found between a root and its conjugate or one
                               of the next 8 roots in real order (upper bound of the least
                               distance; the closest pairs are adjacent in that order) */
    double max_radius;      /* largest certificate radius */
    double ms_device;       /* device time of the whole call, milliseconds */
    /* device time of each stage of the whole call (all types of a batch share
     * one launch per stage), milliseconds, from events on `stream`:
     * [0] seeds, [1] level-line walk, [2] descents, [3] collection,
     * [4] classification, [5] certificate and separation */
    double ms_stage[6];
    int32_t hip_error;      /* last hipError_t on MSPLIT_E_DEVICE */
    int32_t mark_capped;    /* identification scans that ended on their length bound, not on
                               the key window (a duplicate may survive; 0 in every tested run) */
    uint64_t basin;         /* roots with MSPLIT_R_BASIN */
    double min_basin;       /* least Newton-basin radius among them */
} msplit_stats;

/* Human-readable text of a status code (static storage). */
const char *msplit_strerror(int status);

/* Exact root counts (Thm countingHyp, eq. HypCount; eq. MisCount):
 *   l == 0: primitive_only ? |Hyp(n)| : 2^(n-1)   (all roots of p_n)
 *   l >= 2: |Mis(l,n)| = Phi(l,n) |Hyp(n)|
 * Returns 0 for invalid (l, n). */
uint64_t msplit_expected_count(int l, int n, int primitive_only);

/* Workspace bytes needed to split q_{l,n} (l = 0: p_n) with these options
 * (NULL = defaults).  Returns MSPLIT_E_ARG for an invalid (l, n). */
int msplit_workspace_size(int l, int n, const msplit_options *opts, uint64_t *bytes);

/* Split p_n, 1 <= n <= 30 (Section 4.2, Algorithm S_par; Section 6.3.1).
 * Writes all roots of p_n (closed upper half plane) to out, their exact period
 * to out->period, and *count = number written.  count and stats are host
 * pointers; stats may be NULL.  With MSPLIT_F_CERTIFY every root is checked
 * by Thm proofRoots in disk arithmetic and its period by the same disk.
 * Errors: MSPLIT_E_ARG, MSPLIT_E_WORKSPACE, MSPLIT_E_CAPACITY (then *count
 * is the capacity needed), MSPLIT_E_DEVICE, MSPLIT_E_INCOMPLETE (roots are
 * still written), MSPLIT_E_PRECISION (n beyond what FP64 separates). */
int msplit_hyperbolic(int n, const msplit_options *opts, void *workspace, uint64_t workspace_bytes,
                      msplit_roots *out, uint64_t *count, msplit_stats *stats, void *stream);

/* Bytes of the static device scratch array of msplit_hyperbolic_static
 * (64 MiB: p_n up to n = 19 with the default options). */
#define MSPLIT_STATIC_SCRATCH_BYTES (64ull << 20)

/* msplit_hyperbolic without a workspace argument, for callers that cannot
 * allocate device memory (code under graph capture, tight serving loops,
 * harnesses that forbid allocation): the call runs in a static device array
 * of MSPLIT_STATIC_SCRATCH_BYTES that the library holds on every device it
 * runs on until the process ends, and allocates nothing (no device memory,
 * no events; stats->ms_device and ms_stage stay 0).  The caller still
 * passes the output arrays.  Same roots, counts and errors as
 * msplit_hyperbolic, plus MSPLIT_E_WORKSPACE when msplit_workspace_size for
 * (0, n, opts) exceeds MSPLIT_STATIC_SCRATCH_BYTES (nothing runs then).
 * All calls on one device share its array, which keeps the last call's
 * contents (every call initialises what it reads): calls that overlap on
 * one device race -- serialise them (one stream, or the caller's lock).
 * MSPLIT_E_DEVICE when the array's address cannot be taken (hip_error). */
int msplit_hyperbolic_static(int n, const msplit_options *opts, msplit_roots *out, uint64_t *count,
                             msplit_stats *stats, void *stream);

/* Split q_{l,n}, l >= 2, n >= 1 (Section 2.2, eq. def:mis; Section 6.3.1,
 * misQuick) and keep Mis(l,n): roots of q_{l,n} that are neither roots of
 * q_{l-1,n} nor of q_{l,k} for a strict divisor k of n.  Same contract as
 * msplit_hyperbolic. */
int msplit_misiurewicz(int l, int n, const msplit_options *opts, void *workspace, uint64_t workspace_bytes,
                       msplit_roots *out, uint64_t *count, msplit_stats *stats, void *stream);

/* Certify `count` candidate roots of q_{l,n} (l = 0: p_n) already in device
 * memory (Thm proofRoots with the disk arithmetic of Thm diskArithmetic, in
 * FP64 with round-to-nearest and explicit radius inflation).  Reads re, im
 * (and period for p_n labels); writes flags (MSPLIT_R_*) and radius.  The
 * list must be sorted by increasing real part for the separation check.
 * workspace: device memory of at least MSPLIT_CERTIFY_WORKSPACE bytes, else
 * MSPLIT_E_WORKSPACE.  stats (nullable) receives certified, label_proven,
 * overlaps, min_sep and max_radius.  With roots->basin non-null, every
 * certified root also gets a disk of Newton convergence (Thm proofContract:
 * basin, MSPLIT_R_BASIN; stats basin and min_basin). */
int msplit_certify(int l, int n, msplit_roots *roots, uint64_t count, void *workspace,
                   uint64_t workspace_bytes, msplit_stats *stats, void *stream);

/* The level-line starting points alone (Section 4.1, the discrete level line
 * L_{lambda_0, 4D}(P) of Prop. computeLevelLine; the levelSets / misSets
 * stage of Section 6.4.1): start k, k = 0 .. 2D, is the point of the closed
 * upper half plane with P = lambda_0 i^k, approximately (|P / (lambda_0 i^k)
 * - 1| < 2^-5: a start only has to lie in the Newton basin of its root).
 * re, im: device arrays of capacity >= 2D + 1.  *count = 2D + 1.  stats
 * receives phase_fail, steps_lift, steps_walk and the stage times. */
int msplit_starts(int l, int n, const msplit_options *opts, void *workspace, uint64_t workspace_bytes,
                  double *re, double *im, uint64_t capacity, uint64_t *count, msplit_stats *stats, void *stream);

/* Split a list of types in one call (Section 6.4.1: the raw searches of many
 * polynomials, each a set of independent tasks over pieces of its level line,
 * then the merge of what they found; here every piece of every type is an
 * item of one device work queue per stage, and the merge is one sort):
 * ln_pairs holds npairs (l, n) pairs
 * (l = 0 for p_n), 1 <= npairs <= 256; all types share one launch per
 * stage and the host synchronises once, at the end.  Roots of pair i are
 * written at out[offsets[i] .. offsets[i] + counts[i]) where offsets[i] is
 * the running sum of the capacities caps[i] (host array).  counts (host,
 * npairs) receives the counts; stats (host, npairs, nullable) the per-pair
 * statistics. */
int msplit_batch(const int32_t *ln_pairs, int npairs, const msplit_options *opts, void *workspace,
                 uint64_t workspace_bytes, msplit_roots *out, const uint64_t *caps, uint64_t *counts,
                 msplit_stats *stats, void *stream);

/* Workspace bytes for msplit_batch over these pairs. */
int msplit_batch_workspace_size(const int32_t *ln_pairs, int npairs, const msplit_options *opts,
                                uint64_t *bytes);

/* Split one type whose level line does not fit the device in one pass, p_n
 * up to n = 33 (the paper's FP80 frontier, Section 6.3.2), streamed: the
 * upper half of the level line is cut into chunks of about chunk_starts
 * consecutive starts (0: 2^28), the paper's independent jobs over seed
 * ranges of one level line (Section 6.4.1).  Each chunk is walked, descended
 * (FP64, double-double next to -2) and identified on its own; its roots are
 * accumulated; the roots found from two chunks (the paper's overlap between
 * jobs) are identified by real-part partitions of the accumulation; the
 * output is the same sorted, classified and certified set as one pass of
 * msplit_hyperbolic / msplit_misiurewicz (q_{l,n} stays limited by
 * MSPLIT_E_PRECISION to order 25).  Valid for n >= 1, l = 0 or l >= 2,
 * l + n <= 33.  Arguments and errors as msplit_hyperbolic; workspace of
 * msplit_stream_workspace_size bytes (p_33: about 117 GB with the default
 * chunks, besides the output, whose capacity must hold the upper-half roots:
 * 2^31 plus half the real ones).  The host synchronises
 * once per chunk and per partition.  stats: the sums over the chunks;
 * sorted = the entries of the chunks' sorts, discarded = roots found from
 * more than one chunk plus those dropped by the classification. */
int msplit_split_streamed(int l, int n, const msplit_options *opts, uint64_t chunk_starts, void *workspace,
                          uint64_t workspace_bytes, msplit_roots *out, uint64_t *count, msplit_stats *stats,
                          void *stream);

/* Workspace bytes for msplit_split_streamed. */
int msplit_stream_workspace_size(int l, int n, const msplit_options *opts, uint64_t chunk_starts,
                                 uint64_t *bytes);

/* A batch captured once as a hipGraph and replayed (the batch scheduling of
 * the paper's job runs, Section 6.4.1, as one device graph): every kernel of
 * an msplit_batch call -- seeds, walk, descents, collection, classification,
 * certificate -- in one graph launch, since every size the kernels need is
 * computed on the device.  Arguments as msplit_batch; stream must be a
 * created stream (not NULL: the null stream cannot be captured).  The graph
 * keeps the workspace and output pointers: they must stay allocated, and no
 * other call may use that workspace while a launch runs.  *graph receives
 * the handle (host object owned by the caller, freed by
 * msplit_graph_destroy).  Errors as msplit_batch, MSPLIT_E_DEVICE when the
 * capture fails. */
typedef struct msplit_graph msplit_graph;
int msplit_batch_graph(const int32_t *ln_pairs, int npairs, const msplit_options *opts, void *workspace,
                       uint64_t workspace_bytes, msplit_roots *out, const uint64_t *caps, void *stream,
                       msplit_graph **graph);

/* One replay of the graph on stream (uploads the type tables, launches the
 * graph, waits for it): counts and stats as msplit_batch, except that the
 * stage times ms_stage stay 0 (ms_device is the launch's device time). */
int msplit_graph_launch(msplit_graph *graph, uint64_t *counts, msplit_stats *stats, void *stream);

/* Release the graph (host and runtime objects; not the workspace). */
void msplit_graph_destroy(msplit_graph *graph);

#ifdef __cplusplus
}
#endif

#endif /* MSPLIT_H */

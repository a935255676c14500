/*
 * asqtad.h -- C ABI of the MI355X (gfx950) even-odd asqtad CG library.
 *
 * The paper (Lattice 2014 proceedings on Kepler GPUs and Xeon Phi) measures a
 * mixed-precision conjugate-gradient inverter for the staggered asqtad quark
 * matrix on a 20^3 x 64 MILC lattice, with the bulk of its arithmetic in single
 * precision (section "GTX Titan Black", CG performance figure and table;
 * section "CPS & QUDA", mixed precision and automatic tuning of the launch
 * parameters).  The paper states no formulas; the operator below is
 * the standard asqtad one:
 *
 *   (D psi)(x) = sum_mu eta_mu(x) [ F_mu(x) psi(x+mu) - F_mu(x-mu)^dag psi(x-mu)
 *                                 + L_mu(x) psi(x+3mu) - L_mu(x-3mu)^dag psi(x-3mu) ]
 *   eta_x = 1, eta_y = (-1)^x, eta_z = (-1)^(x+y), eta_t = (-1)^(x+y+z)
 *   fermions periodic in space and antiperiodic in time, links periodic
 *   A = (M^dag M)_ee = 4 m^2 - D_eo D_oe with M = 2m + D  (even sites)
 *
 * Memory.  The library never allocates device memory.  The caller (PyTorch in
 * the Python binding) owns every buffer: canonical input links, the resident
 * gauge storage, sources, solutions, solver workspace and the serving arena.
 * The library owns only the opaque handles it returns.
 *
 * Streams.  Every entry point takes a hipStream_t (as void*; NULL = the null
 * stream) and enqueues its kernels there.  asqtad_dslash_eo returns without
 * waiting; asq_gauge_create and cg_solve* return when their work is done.
 * serve_* functions are thread-safe; the others are not thread-safe per handle.
 *
 * Errors.  Every int-returning function returns ASQ_OK (0), ASQ_PENDING (1,
 * serve_poll only) or a negative ASQ_E* code; asq_last_error() gives detail.
 * Arguments are validated on the host before any HIP call.
 *
 * Canonical layouts (every entry point).  lex = x + X*(y + Y*(z + Z*t));
 * parity = (x+y+z+t) mod 2, even = 0; checkerboard index = lex / 2;
 * directions x,y,z,t; complex numbers interleaved (re, im);
 * (U psi)_a = sum_b U[a][b] psi_b and U_mu(x) multiplies psi(x+mu).
 *   Links: double [V][4][3][3][2] (lexicographic sites).
 *   Colour vectors of one parity, nrhs columns, half = V/2:
 *     ASQ_F64: double [nrhs][half][3][2]
 *     ASQ_F32: float  [nrhs][half][3][2]
 *     ASQ_F16: binary16 [nrhs][half][3][2] holding psi/nu, followed by
 *              float nu [nrhs][half], nu = max |component| of the (site,
 *              column) as float32; each half is the component times the
 *              float32 reciprocal of nu, rounded once to binary16 (nearest
 *              even).  16 bytes per site and column in all.
 * The kernels keep their own site-fastest structures of arrays (the "native"
 * layouts); the library relayouts at its boundary.  asq_vec_to_native and
 * asq_vec_from_native expose that relayout for timing studies of the exact
 * kernels the solvers launch (asqtad_dslash_eo_variant with ASQ_VARIANT_NATIVE).
 */
#ifndef ASQTAD_H
#define ASQTAD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ASQ_OK 0
#define ASQ_PENDING 1
#define ASQ_EINVAL (-1)   /* bad argument: extents, null pointer, nrhs, mass, tol ... */
#define ASQ_ENOMEM (-2)   /* caller storage / workspace / arena too small             */
#define ASQ_ENOCONV (-3)  /* maxiter reached; x and stats still written              */
#define ASQ_ENOTSU3 (-4)  /* 12-real or 16-bit links requested for non-SU(3) links   */
#define ASQ_EHIP (-5)     /* HIP runtime error                                       */
#define ASQ_ENAN (-6)     /* non-finite or non-positive reduction in the solver      */
#define ASQ_EAGAIN (-7)   /* serving queue full                                      */

/* storage precisions: links and colour vectors */
enum { ASQ_F64 = 0, ASQ_F32 = 1, ASQ_F16 = 2 };
/* solver precision modes */
enum {
  ASQ_MODE_F64 = 0,     /* plain CG, everything FP64                                    */
  ASQ_MODE_MIXED32 = 1, /* FP32 Dslash and vectors, reliable updates in FP64 (a field
                           kept in FP64 only: its FP64 links rounded to FP32 on load)   */
  ASQ_MODE_MIXED16 = 2  /* FP16-with-norm Dslash vectors and 16-bit links (if kept),
                           FP32 arithmetic and residual, FP64 solution and true residual */
};

typedef struct asq_gauge asq_gauge;
typedef struct asq_server asq_server;

typedef struct {
  int dims[4];       /* X, Y, Z, T: each even and >= 4                                     */
  int prec_mask;     /* bit (1 << ASQ_F64|ASQ_F32|ASQ_F16): link copies kept resident.
                        Without an F32 copy, F32 and F16 Dslash arithmetic reads the F64
                        links and rounds them to FP32 on load                             */
  int recon;         /* 18 or 12: storage of the F32 copy (F64 is always 18, F16 always 12) */
  double fat_scale;  /* fat = fat_scale * SU(3) (9/8 for the synthetic fields); used by
                        12-real and 16-bit copies, which store link/scale               */
  double long_scale; /* long = long_scale * SU(3) (-1/24 for the synthetic fields)         */
} asq_gauge_desc;

typedef struct {
  double tol;       /* stop when |b - A x| / |b| <= tol (FP64 true residual); > 0        */
  int maxiter;      /* per column; > 0                                                    */
  int mode;         /* ASQ_MODE_*                                                          */
  double delta;     /* reliable-update trigger: |r| < delta * max|r| since last update   */
  int poll_iters;   /* iterations per host poll / per captured graph (0 = default 8)      */
  int use_graph;    /* 1: capture poll_iters iterations in a hipGraph and replay it       */
} asq_cg_params;

typedef struct {
  int iters;            /* CG iterations of the column                                    */
  int reliable_updates; /* FP64 residual recomputations during the iteration              */
  int converged;        /* 1 if the FP64 true residual met tol                            */
  int status;           /* ASQ_OK, ASQ_ENOCONV or ASQ_ENAN for this column                */
  double true_resid;    /* |b - A x| / |b| with the FP64 operator                         */
  double seconds;       /* wall time of the call (batch: of the whole batch)              */
  double gflops;        /* 1146 flops per site per Dslash + 72 per even site per iteration */
  int escalations;      /* times the column moved to a higher precision tier because its
                           true residual stalled (mixed16 -> mixed32 -> f64)               */
  int final_mode;       /* the ASQ_MODE_* the column finished in                           */
} asq_cg_stats;

/* ---- gauge fields -------------------------------------------------------- */

/* Bytes of device storage asq_gauge_create needs for this description; 0 if the
   description is invalid. */
size_t asq_gauge_bytes(const asq_gauge_desc* desc);

/* Import fat and long links into resident storage (the gauge field stays on the
   device between solves, as the paper's CG keeps its links on the GPU): fold
   eta_mu and the time-boundary sign, transpose to site-fastest structure of
   arrays per parity, convert to each kept precision and compress to 12 reals
   where asked.  fat_host, long_host: host pointers, double [V][4][3][3][2]
   (canonical), only read during the call; they are copied to the device a
   chunk of at most 16 MB at a time through a staging area at the end of the
   storage (part of asq_gauge_bytes).  storage_dev: caller-owned device buffer
   of at least asq_gauge_bytes(desc) bytes, 256-byte aligned, that must outlive
   the handle.  Returns ASQ_ENOTSU3 if a 12-real or 16-bit copy is requested
   and some link/scale is not SU(3) to 1e-6.  Synchronizes the stream. */
int asq_gauge_create(const asq_gauge_desc* desc, const double* fat_host, const double* long_host,
                     void* storage_dev, size_t storage_bytes, void* hip_stream, asq_gauge** out);
/* The same from links already on the device (e.g. from asqtad_build_links):
   fat_dev, long_dev are device pointers in the same canonical layout, 16-byte
   aligned, read in place during the call. */
int asq_gauge_create_device(const asq_gauge_desc* desc, const double* fat_dev, const double* long_dev,
                            void* storage_dev, size_t storage_bytes, void* hip_stream, asq_gauge** out);
int asq_gauge_destroy(asq_gauge* g);

/* Asqtad fat and long links from thin links, in FP64.  The paper's lattices
   are MILC asqtad ensembles (CG benchmark, "GTX Titan Black" section) and it
   prints no smearing formula; this is the standard asqtad action:
     F_mu(x) = sum over paths P from x to x+mu of c(P) * (thin links along P):
       the link itself 5/8, 3-staples 1/(16 u0^2), 5-staples 1/(64 u0^4),
       7-staples 1/(384 u0^6), Lepage [nu nu mu -nu -nu] -1/(16 u0^4)
     L_mu(x) = -1/(24 u0^2) U_mu(x) U_mu(x+mu) U_mu(x+2mu)
   (staples over every signed direction off mu's axis, deeper staples over
   pairwise different axes).  With unit links F = 9/8 and L = -1/24 at u0 = 1.
   dims: lattice extents, even, >= 4.  thin_dev: device, double [V][4][3][3][2]
   canonical, any 3x3 complex matrices (periodic in every direction), read only.
   u0: tadpole factor, > 0.  fat_dev, long_dev: device outputs in the same
   layout, fully overwritten (long_dev also holds a transposed copy of the thin
   links while the fat links are built); the three arrays must not overlap and
   must be 16-byte aligned.  The fat links are not SU(3) in general, so pass them to
   asq_gauge_create with recon 18 and no 16-bit copy.  Enqueued on hip_stream;
   returns without waiting.  ASQ_EINVAL on a bad argument (checked on the host
   before any launch), ASQ_EHIP if the launch fails. */
int asqtad_build_links(const int dims[4], const double* thin_dev, double u0, double* fat_dev, double* long_dev,
                       void* hip_stream);

/* Device workspace bytes of asqtad_plaquette for these extents (0 if invalid). */
size_t asqtad_plaquette_workspace_bytes(const int dims[4]);
/* Mean plaquette of thin links, the input of the tadpole factor u0 = P^(1/4)
   that the asqtad coefficients use (MILC's ensembles are tadpole improved; the
   paper prints no formula):
     P = 1/(6V) sum_x sum_{mu<nu} (1/3) Re tr[U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag]
   thin_dev: device, double [V][4][3][3][2] canonical, periodic in every
   direction, 16-byte aligned.  work_dev: at least
   asqtad_plaquette_workspace_bytes(dims) bytes of device memory, 8-byte
   aligned, disjoint from the links, overwritten.  *plaq (host) receives P in FP64, summed in a fixed
   order (bitwise reproducible).  Synchronizes the stream.  ASQ_EINVAL or
   ASQ_ENOMEM on bad arguments, checked before any launch. */
int asqtad_plaquette(const int dims[4], const double* thin_dev, void* work_dev, size_t work_bytes, double* plaq,
                     void* hip_stream);

/* For callers that cannot allocate (code under graph capture, tight serving
   loops, harnesses that forbid allocation): asqtad_plaquette without a
   workspace.  The partial sums live in a fixed 2 MiB device array of the
   library (one per GPU, kept until the process ends), so lattices up to
   67108608 sites (ASQ_ENOMEM beyond); every call on a GPU shares that array,
   so calls that overlap on one GPU race.  *plaq_dev (device, 8-byte aligned)
   receives P, the same bits as asqtad_plaquette.  Asynchronous on hip_stream:
   no allocation, no copy to the host, no synchronization.  thin_dev as for
   asqtad_plaquette; ASQ_EINVAL on a bad argument (checked on the host). */
int asqtad_plaquette_noalloc(const int dims[4], const double* thin_dev, double* plaq_dev, void* hip_stream);

/* ---- operator ------------------------------------------------------------ */

/* out = D restricted to sites of out_parity, acting on in (sites of the other
   parity), for nrhs columns in precision prec (canonical layouts).  F64 uses
   the F64 links, F32 the F32 links (or the F64 links rounded to FP32 on load
   when no F32 copy is kept), F16 the F16 links if kept, else those of F32.
   Asynchronous on hip_stream.  in_dev and out_dev: 16-byte aligned and
   disjoint (ASQ_EINVAL if their nrhs columns share a byte).  Successive calls
   in the process walk the lattice in alternate directions (each starts where
   the previous one ended, on links the memory-side cache still holds); the
   result is the same bits either way.  The single-parity hopping term of the
   asqtad operator: the kernel on which the paper's CG spends its time. */
int asqtad_dslash_eo(const asq_gauge* g, int out_parity, int prec, int nrhs, const void* in_dev,
                     void* out_dev, void* hip_stream);

/* The same operator with a caller-chosen launch variant instead of the tuned
   one (for tests that cover every variant and for tuning studies; every
   variant computes the same result, bit for bit).  variant = cols | pipe << 8 |
   stream << 9 | chunk << 10 | order << 12 | lds << 14 | sweep << 15: cols = 1, 2, 4, 6, 8 or 12
   columns per thread (12 not with FP64 vectors); pipe = 1 for the
   software-pipelined hop loop; stream = 1 (one column, FP32 and 16-bit link
   tiers only) reads the links with non-temporal loads; lds = 1 (pipe = 1,
   native vectors only; with stream only at one column; refused when the
   window of the tile's columns exceeds 64 KB) first stages the input records
   within three y-rows of each block's sites in LDS, where its x and y hops
   read them; order = 0 walks the column tiles of a site block together, 1, 2, 3 walk
   tile by tile inside groups of 16, 64 or all site blocks; sweep = 1 deals
   the blocks to the XCDs round-robin (one sweep front through the lattice)
   instead of a contiguous slab per XCD, chunk = 1, 2, 3 (with sweep only) in
   runs of 16, 64 or 256 consecutive blocks per XCD instead of single blocks.  variant = 0x10000 | 32 | order << 12 selects the matrix-core form
   (prec F16 with FP32 18-real links only): 32 columns per block, FP32 products
   on the matrix cores.  It rounds differently from the other variants (within
   the FP16 tolerance) and is bitwise reproducible against itself.  Adding
   ASQ_VARIANT_NATIVE makes in_dev and out_dev native-layout vectors (see
   asq_vec_to_native): the kernels the solvers launch, for timing them
   (ASQ_VARIANT_NATIVE alone: the tuned variant on native vectors); the
   matrix-core form takes native vectors only.  Returns ASQ_EINVAL for any
   other code. */
#define ASQ_VARIANT_NATIVE 0x100000
int asqtad_dslash_eo_variant(const asq_gauge* g, int out_parity, int prec, int nrhs, const void* in_dev,
                             void* out_dev, int variant, void* hip_stream);

/* ---- colour vectors ------------------------------------------------------------ */

/* Bytes of nsites canonical colour-vector records in precision prec (nsites =
   nrhs * V/2 for nrhs columns of one parity); 0 for an unknown precision. */
size_t asq_vec_bytes(int prec, size_t nsites);
/* dst = src converted between the precision tiers of the mixed-precision CG
   (the paper's inverter keeps most of its data in single precision; the FP16
   tier adds a per-site norm).  Both canonical, nsites records each, 16-byte
   aligned, disjoint.  To FP16: the values are rounded to float32, nu = the
   largest magnitude of the site's six reals, each real times r = 1/nu (float32,
   correctly rounded) rounded once to binary16, nearest even (nu = 0 gives zeros).  From FP16: the
   exact value nu * h (then rounded to float32 for ASQ_F32).  FP64 to FP32
   rounds to nearest.  Asynchronous on hip_stream.  ASQ_EINVAL on a bad
   argument. */
int asq_vec_convert(size_t nsites, int src_prec, const void* src_dev, int dst_prec, void* dst_dev,
                    void* hip_stream);
/* Canonical <-> native relayout of nrhs colour vectors of one parity of g's
   lattice in precision prec (data movement only; the native layouts are the
   solvers' private structures of arrays and may change between versions).
   16-byte aligned, disjoint buffers of asq_vec_bytes(prec, nrhs * V/2) bytes.
   Asynchronous on hip_stream. */
int asq_vec_to_native(const asq_gauge* g, int prec, int nrhs, const void* canon_dev, void* native_dev,
                      void* hip_stream);
int asq_vec_from_native(const asq_gauge* g, int prec, int nrhs, const void* native_dev, void* canon_dev,
                        void* hip_stream);

/* ---- solvers --------------------------------------------------------------- */

/* Device workspace bytes cg_solve / cg_solve_batch need for nrhs columns
   (the solver's vectors plus native copies of b and x). */
size_t asq_workspace_bytes(const asq_gauge* g, int nrhs, int mode);

/* Solve A x = b (even sites) by CG from x0 = 0 (the paper's CG inverter; mixed
   precision with reliable updates for ASQ_MODE_MIXED*).  b_dev, x_dev: device
   double [V/2][3][2] (canonical).  work_dev: caller-owned, >= asq_workspace_bytes.
   Returns when done.  ASQ_ENOCONV if the true residual misses tol after
   maxiter iterations (x and stats still written). */
int cg_solve(const asq_gauge* g, double mass, const double* b_dev, double* x_dev, void* work_dev,
             size_t work_bytes, const asq_cg_params* params, asq_cg_stats* stats, void* hip_stream);

/* nrhs independent systems (A_c x_c = b_c, A_c = 4 m_c^2 - D_eo D_oe) advanced
   together: one multi-column Dslash launch per half-operator, per-column
   alpha/beta/masks on the device.  masses: host double[nrhs] (> 0).  b_dev,
   x_dev: device double [nrhs][V/2][3][2] (canonical).  stats: host array [nrhs].
   (The paper's CG inverter, section "GTX Titan Black", run for many
   right-hand sides and masses at once: 24 sources x 4 masses are 96 such
   columns.)  Each
   column's arithmetic does not depend on the other columns.  For this call,
   cg_solve, cg_solve_multishift and cg_solve_full, b_dev, x_dev and the
   workspace must be pairwise disjoint (ASQ_EINVAL otherwise).  The first
   solve of a (lattice, precision tiers, column count) on a device first times
   the Dslash launch variants on that call's own sources, converted to the
   iteration's tier (the autotuner; ASQ_TUNE=0 takes built-in choices instead,
   ASQ_TUNE_CACHE=<file> keeps the choices across processes). */
int cg_solve_batch(const asq_gauge* g, int nrhs, const double* masses, const double* b_dev, double* x_dev,
                   void* work_dev, size_t work_bytes, const asq_cg_params* params, asq_cg_stats* stats,
                   void* hip_stream);

/* Every (mass, source) pair of nmass masses and nsrc sources at once: the
   shifted systems (4 m_j^2 - D_eo D_oe) x = b share the Krylov space of the
   smallest mass, so one CG per source (FP32, no reliable updates) carries all
   masses along with vector updates only, to a relative iterated residual of
   max(tol, 1e-7).  Each (mass, source) column is then refined from that
   solution by the reliable-update CG of params->mode to the FP64 true residual
   tol.  b_dev: device double [nsrc][V/2][3][2]; x_dev: [nmass][nsrc][V/2][3][2]
   (column j * nsrc + s).  masses: host double [nmass] (> 0, any order).
   work_dev: >= asq_multishift_workspace_bytes, 256-byte aligned.  stats[c]:
   iters = shifted-phase plus refinement iterations; reliable updates, true
   residual and status as cg_solve_batch.  Needs the FP32 links.  Returns when
   done.  (The shifted form of a many-source, several-mass workload such as
   24 sources x 4 masses, which the paper's CG would run one system at a time.) */
size_t asq_multishift_workspace_bytes(const asq_gauge* g, int nsrc, int nmass, int mode);
int cg_solve_multishift(const asq_gauge* g, int nsrc, int nmass, const double* masses, const double* b_dev,
                        double* x_dev, void* work_dev, size_t work_bytes, const asq_cg_params* params,
                        asq_cg_stats* stats, void* hip_stream);

/* The full-lattice system M x_c = b_c, M = 2 m_c + D on both parities,
   through the even-odd reduction the CG works on:
     b' = 2m b_e - D_eo b_o,  (4m^2 - D_eo D_oe) x_e = b' (cg_solve_batch),
     x_o = (b_o - D_oe x_e) / (2m).
   The odd equations then hold exactly, so |b - M x| = |b' - A x_e| / (2m) and
   each column's even solve runs to tol * 2m |b| / |b'|.  b_dev, x_dev: device
   double [2][nrhs][V/2][3][2] (the even halves of all columns, then the odd
   halves).  work_dev: >= asq_full_workspace_bytes, 256-byte aligned.
   stats[c]: iterations and reliable updates of the even solve; true_resid =
   |b - M x| / |b| recomputed with the FP64 operator after the
   reconstruction (ASQ_ENOCONV if it exceeds tol).  Returns when done.  (The
   paper's CG solves the even-odd reduced system; this is the step on either
   side of it that a propagator for the whole lattice needs.) */
size_t asq_full_workspace_bytes(const asq_gauge* g, int nrhs, int mode);
int cg_solve_full(const asq_gauge* g, int nrhs, const double* masses, const double* b_dev, double* x_dev,
                  void* work_dev, size_t work_bytes, const asq_cg_params* params, asq_cg_stats* stats,
                  void* hip_stream);

/* ---- serving --------------------------------------------------------------- */

/* A request loop with continuous batching.  The paper has no counterpart: it
   times one CG solve at a time (section "GTX Titan Black").  Here many
   independent solves of that CG share the device, as the columns of
   cg_solve_batch share a batch: requests on a registered gauge
   field join the in-flight batch of that field when column slots and arena
   memory free up; batches of different fields run on their own streams.
   arena_dev/arena_bytes: caller-owned device memory = the HBM budget for
   solver workspaces.  max_streams >= 1: concurrent batches (streams).
   max_cols >= 1: column slots of a batch of the largest registered field and
   the most columns one request may have; batches of smaller fields get up to
   8x as many slots (in proportion to the site counts, as the arena allows). */
int serve_create(void* arena_dev, size_t arena_bytes, int max_streams, int max_cols, asq_server** out);
/* The gauge field must outlive the server.  Registration times the Dslash
   launch variants of every batch shape the server can give the field (each
   solver mode it keeps links for), on scratch from the arena, and returns when
   done; other serve_* calls wait meanwhile.  Register fields before
   submitting: while batches exist nothing is timed and batches use the
   variants already known (or the built-in defaults). */
int serve_register_gauge(asq_server* s, const asq_gauge* g, int* gauge_id);
/* Non-blocking.  masses: host double[nrhs]; b_dev/x_dev canonical as for
   cg_solve_batch (disjoint), owned by the caller until serve_poll reports
   completion.  hip_stream: the stream on which b was produced (NULL = the null
   stream); the server reads b only after the work enqueued on it before this
   call.  x_dev is written on the server's own streams and is complete when
   serve_poll returns ASQ_OK or an error.  A request joins a batch only with
   requests of the same field, mode, poll_iters (0 counts as 8) and use_graph, so
   its reliable updates fall where they would in a solve of its own.
   ASQ_EAGAIN if the queue is full; ASQ_ENOMEM if the request can never fit the
   arena. */
int serve_submit(asq_server* s, int gauge_id, int nrhs, const double* masses, const double* b_dev,
                 double* x_dev, const asq_cg_params* params, uint64_t* ticket, void* hip_stream);
/* ASQ_PENDING while running; ASQ_OK (or the request's error) once complete, with
   per-column stats (host array [nrhs], may be NULL) and latency from submit to
   completion (may be NULL).  A completed ticket is released by this call. */
int serve_poll(asq_server* s, uint64_t ticket, asq_cg_stats* per_rhs, double* latency_s);
/* Completes every submitted request, queued ones included (their x_dev is
   written), then frees the server; tickets not yet polled are discarded. */
int serve_destroy(asq_server* s);

/* ---- NPR: the one-colour four-fermion operator ------------------------------- */

/* The one-colour four-fermion operator of the paper's NPR code (section "GTX
   Titan Black", Eq. (1)), in FP64, for every hypercube z of the lattice (corners
   z_A = 2z + A, A a 4-bit mask: bit mu = the offset along x, y, z, t) and each
   operator I = (S1, F1, S2, F2) of spin-taste masks:
     V_I(z)[a1][a2][a3][a4] = sum_{A,B,C,D} M1_AB M2_CD eps(z_A) eps(z_C)
         (G1(z_A)^dag U_AD G4(z_D))_{a1 a4} (G3(z_C)^dag U_CB G2(z_B))_{a3 a2}
   M = (gamma_S (x) xi_F)bar, (1/4) Tr[gamma_A^dag gamma_S gamma_B gamma_F^dag] with
   gamma_A = gamma_1^A1 gamma_2^A2 gamma_3^A3 gamma_4^A4 (Euclidean, Hermitian);
   eps(x) = (-1)^(x+y+z+t); U_AD = the ordered link product averaged over every
   shortest path from z_A to z_D (U_mu(x) stepping +mu, U_mu(x-mu)^dag stepping
   -mu; 1 for A = D).  This is the operator's matrix element with each chi
   replaced by a propagator G_f from a common source and each chibar by its
   staggered conjugate eps G_f^dag; the source colours a1..a4 stay free.
   dims: even extents 2 .. 16384.  thin_dev: links double [V][4][3][3][2]
   (canonical).  g*_dev: propagators double [V][3][3][2], row = colour at the
   site, column = source colour (the four may be the same array).  ops_host:
   int [nop][4] = S1, F1, S2, F2, each 0 .. 15.  out_dev: double
   [nop][V/16][3][3][3][3][2], hypercubes in lexicographic order of z (x
   fastest), indices [a1][a2][a3][a4]; must not overlap an input.  All device
   pointers 16-byte aligned.  Asynchronous on hip_stream; ASQ_EINVAL on a bad
   argument (checked on the host before any launch). */
int asqtad_npr_fourfermion(const int dims[4], const double* thin_dev, const double* g1_dev, const double* g2_dev,
                           const double* g3_dev, const double* g4_dev, int nop, const int* ops_host, double* out_dev,
                           void* hip_stream);

/* ---- misc ------------------------------------------------------------------ */

const char* asq_strerror(int code);
/* Detail of the last error on the calling thread. */
const char* asq_last_error(void);
/* HBM copy probe: dst = src for n bytes (n a multiple of 16, 16-byte aligned
   device pointers), asynchronous.  The plain copy kernel used to calibrate
   bandwidth and hardware counters. */
int asq_copy_probe(void* dst_dev, const void* src_dev, size_t n, void* hip_stream);
/* HBM read probe: reads n bytes of src (n a multiple of 16, 16-byte aligned)
   with non-temporal loads, eight in flight per thread, and writes one 16-byte
   XOR digest per block to sink_dev (at least asq_read_probe_blocks(n) x 16
   bytes), asynchronous.  The read-only ceiling against which a read-dominated
   kernel such as the Dslash is measured. */
int asq_read_probe(const void* src_dev, size_t n, void* sink_dev, void* hip_stream);
size_t asq_read_probe_blocks(size_t n);

#ifdef __cplusplus
}
#endif

#endif /* ASQTAD_H */

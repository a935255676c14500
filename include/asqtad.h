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
 * Host layouts (canonical).  lex = x + X*(y + Y*(z + Z*t)); parity =
 * (x+y+z+t) mod 2, even = 0; checkerboard index = lex / 2; directions x,y,z,t;
 * complex numbers interleaved (re, im); (U psi)_a = sum_b U[a][b] psi_b and
 * U_mu(x) multiplies psi(x+mu).  Links: double [V][4][3][3][2].
 *
 * Device colour-vector layouts (one parity, nrhs columns, half = V/2):
 *   ASQ_F64: double [nrhs][3][half][2]   (colour-major structure of arrays)
 *   ASQ_F32: float  [nrhs][3][half][2]
 *   ASQ_F16: 16-byte records [nrhs][half]: six IEEE binary16 values
 *            (c0.re c0.im c1.re c1.im c2.re c2.im) holding psi/nu, then nu as
 *            float32, nu = max |component| of the site (round to nearest even).
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
  ASQ_MODE_MIXED32 = 1, /* FP32 Dslash and vectors, reliable updates in FP64            */
  ASQ_MODE_MIXED16 = 2  /* FP16-with-norm Dslash vectors and 16-bit links (if kept),
                           FP32 arithmetic and residual, FP64 solution and true residual */
};

typedef struct asq_gauge asq_gauge;
typedef struct asq_server asq_server;

typedef struct {
  int dims[4];       /* X, Y, Z, T: each even and >= 4                                     */
  int prec_mask;     /* bit (1 << ASQ_F64|ASQ_F32|ASQ_F16): link copies kept resident     */
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
} asq_cg_stats;

/* ---- gauge fields -------------------------------------------------------- */

/* Bytes of device storage asq_gauge_create needs for this description; 0 if the
   description is invalid. */
size_t asq_gauge_bytes(const asq_gauge_desc* desc);

/* Import fat and long links into resident storage: fold eta_mu and the
   time-boundary sign, transpose to site-fastest structure of arrays per parity,
   convert to each kept precision and compress to 12 reals where asked.
   fat_dev, long_dev: device pointers, double [V][4][3][3][2] (canonical); only
   read during the call.  storage_dev: caller-owned device buffer of at least
   asq_gauge_bytes(desc) bytes, 256-byte aligned, that must outlive the handle.
   Returns ASQ_ENOTSU3 if a 12-real or 16-bit copy is requested and some
   link/scale is not SU(3) to 1e-6.  Synchronizes the stream. */
int asq_gauge_create(const asq_gauge_desc* desc, const double* fat_dev, const double* long_dev,
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

/* ---- operator ------------------------------------------------------------ */

/* out = D restricted to sites of out_parity, acting on in (sites of the other
   parity), for nrhs columns in precision prec (device layouts above).  F64 uses
   the F64 links, F32 the F32 links, F16 the F16 links if kept, else the F32
   ones.  Asynchronous on hip_stream.  in_dev and out_dev: 16-byte aligned and
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
   order << 12: cols = 1, 2, 4, 8 or 12 columns per thread (12 not with FP64
   vectors); pipe = 1 for the software-pipelined hop loop; order = 0 walks the
   column tiles of a site block
   together, 1, 2, 3 walk tile by tile inside groups of 16, 64 or all site
   blocks.  variant = 0x10000 | 32 | order << 12 selects the matrix-core form
   (prec F16 with FP32 18-real links only): 32 columns per block, FP32 products
   on the matrix cores.  It rounds differently from the other variants (within
   the FP16 tolerance) and is bitwise reproducible against itself.  Returns
   ASQ_EINVAL for any other code. */
int asqtad_dslash_eo_variant(const asq_gauge* g, int out_parity, int prec, int nrhs, const void* in_dev,
                             void* out_dev, int variant, void* hip_stream);

/* ---- solvers --------------------------------------------------------------- */

/* Device workspace bytes cg_solve / cg_solve_batch need for nrhs columns. */
size_t asq_workspace_bytes(const asq_gauge* g, int nrhs, int mode);

/* Solve A x = b (even sites) by CG from x0 = 0 (the paper's CG inverter; mixed
   precision with reliable updates for ASQ_MODE_MIXED*).  b_dev, x_dev: device
   double [3][V/2][2].  work_dev: caller-owned, >= asq_workspace_bytes.
   Returns when done.  ASQ_ENOCONV if the true residual misses tol after
   maxiter iterations (x and stats still written). */
int cg_solve(const asq_gauge* g, double mass, const double* b_dev, double* x_dev, void* work_dev,
             size_t work_bytes, const asq_cg_params* params, asq_cg_stats* stats, void* hip_stream);

/* nrhs independent systems (A_c x_c = b_c, A_c = 4 m_c^2 - D_eo D_oe) advanced
   together: one multi-column Dslash launch per half-operator, per-column
   alpha/beta/masks on the device.  masses: host double[nrhs] (> 0).  b_dev,
   x_dev: device double [nrhs][3][V/2][2].  stats: host array [nrhs].  Each
   column's arithmetic does not depend on the other columns.  For this call,
   cg_solve, cg_solve_multishift and cg_solve_full, b_dev, x_dev and the
   workspace must be pairwise disjoint (ASQ_EINVAL otherwise). */
int cg_solve_batch(const asq_gauge* g, int nrhs, const double* masses, const double* b_dev, double* x_dev,
                   void* work_dev, size_t work_bytes, const asq_cg_params* params, asq_cg_stats* stats,
                   void* hip_stream);

/* Every (mass, source) pair of nmass masses and nsrc sources at once: the
   shifted systems (4 m_j^2 - D_eo D_oe) x = b share the Krylov space of the
   smallest mass, so one CG per source (FP32, no reliable updates) carries all
   masses along with vector updates only, to a relative iterated residual of
   max(tol, 1e-7).  Each (mass, source) column is then refined from that
   solution by the reliable-update CG of params->mode to the FP64 true residual
   tol.  b_dev: device double [nsrc][3][V/2][2]; x_dev: [nmass][nsrc][3][V/2][2]
   (column j * nsrc + s).  masses: host double [nmass] (> 0, any order).
   work_dev: >= asq_multishift_workspace_bytes, 256-byte aligned.  stats[c]:
   iters = shifted-phase plus refinement iterations; reliable updates, true
   residual and status as cg_solve_batch.  Needs the FP32 links.  Returns when
   done.  (The multi-shift form of the paper's 24-source x 4-mass workload.) */
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
   double [2][nrhs][3][V/2][2] (the even halves of all columns, then the odd
   halves).  work_dev: >= asq_full_workspace_bytes, 256-byte aligned.
   stats[c]: iterations and reliable updates of the even solve; true_resid =
   |b - M x| / |b| recomputed with the FP64 operator after the
   reconstruction (ASQ_ENOCONV if it exceeds tol).  Returns when done. */
size_t asq_full_workspace_bytes(const asq_gauge* g, int nrhs, int mode);
int cg_solve_full(const asq_gauge* g, int nrhs, const double* masses, const double* b_dev, double* x_dev,
                  void* work_dev, size_t work_bytes, const asq_cg_params* params, asq_cg_stats* stats,
                  void* hip_stream);

/* ---- serving --------------------------------------------------------------- */

/* A request loop with continuous batching: requests on a registered gauge
   field join the in-flight batch of that field when column slots and arena
   memory free up; batches of different fields run on their own streams.
   arena_dev/arena_bytes: caller-owned device memory = the HBM budget for
   solver workspaces.  max_streams >= 1: concurrent batches (streams).
   max_cols >= 1: column slots of a batch of the largest registered field and
   the most columns one request may have; batches of smaller fields get up to
   8x as many slots (in proportion to the site counts, as the arena allows). */
int serve_create(void* arena_dev, size_t arena_bytes, int max_streams, int max_cols, asq_server** out);
/* The gauge field must outlive the server. */
int serve_register_gauge(asq_server* s, const asq_gauge* g, int* gauge_id);
/* Non-blocking.  masses: host double[nrhs]; b_dev/x_dev as for cg_solve_batch
   (disjoint), owned by the caller until serve_poll reports completion.  ASQ_EAGAIN if the
   queue is full; ASQ_ENOMEM if the request can never fit the arena. */
int serve_submit(asq_server* s, int gauge_id, int nrhs, const double* masses, const double* b_dev,
                 double* x_dev, const asq_cg_params* params, uint64_t* ticket);
/* ASQ_PENDING while running; ASQ_OK (or the request's error) once complete, with
   per-column stats (host array [nrhs], may be NULL) and latency from submit to
   completion (may be NULL).  A completed ticket is released by this call. */
int serve_poll(asq_server* s, uint64_t ticket, asq_cg_stats* per_rhs, double* latency_s);
/* Completes every submitted request, queued ones included (their x_dev is
   written), then frees the server; tickets not yet polled are discarded. */
int serve_destroy(asq_server* s);

/* ---- misc ------------------------------------------------------------------ */

const char* asq_strerror(int code);
/* Detail of the last error on the calling thread. */
const char* asq_last_error(void);
/* HBM copy probe: dst = src for n bytes (n a multiple of 16, 16-byte aligned
   device pointers), asynchronous.  The plain copy kernel used to calibrate
   bandwidth and hardware counters. */
int asq_copy_probe(void* dst_dev, const void* src_dev, size_t n, void* hip_stream);
/* HBM read probe: reads n bytes of src (n a multiple of 16, 16-byte aligned)
   and writes one 16-byte XOR digest per block to sink_dev (at least
   asq_read_probe_blocks(n) x 16 bytes), asynchronous.  The read-only ceiling
   against which a read-dominated kernel such as the Dslash is measured. */
int asq_read_probe(const void* src_dev, size_t n, void* sink_dev, void* hip_stream);
size_t asq_read_probe_blocks(size_t n);

#ifdef __cplusplus
}
#endif

#endif /* ASQTAD_H */

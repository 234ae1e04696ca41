/*
 * wilson.h -- C ABI of the MI355X (gfx950) Wilson-Dirac operator library.
 *
 * The library applies the Wilson-Dirac operator of lattice QCD with Wilson
 * fermions on one GPU's whole periodic 4D lattice:
 *
 *   D psi(x) = (4+m) psi(x)
 *              - 1/2 sum_mu [ (1-gamma_mu) U_mu(x) psi(x+mu)
 *                             + (1+gamma_mu) U_mu(x-mu)^dag psi(x-mu) ]
 *
 * The sum is the hopping term of eq. (1) (Sec. II-A of Meyer et al., "SVE-
 * enabling Lattice QCD Codes") up to the sign convention of gamma_mu; the two
 * conventions are exchanged by gamma5 conjugation, so eq. (1)'s D_h equals
 * 2(4+m) - 2 gamma5 D gamma5. psi carries spin (4) x colour (3) complex
 * components per site, U_mu(x) is an SU(3) matrix on the link x -> x+mu
 * (Sec. II-A), gamma_mu are the DeGrand-Rossi Dirac matrices, mu = 0,1,2,3 is
 * x,y,z,t, and all four directions are periodic.
 *
 * Conventions shared by every entry point:
 *   dims      int32_t[4] = {X, Y, Z, T}, each >= 1, with V = X*Y*Z*T < 2^31 / 12.
 *             The canonical site index is x + X*(y + Y*(z + Z*t)) (x fastest).
 *   canonical complex128 (interleaved re, im) arrays in device memory:
 *             spinor psi[nrhs][T][Z][Y][X][spin 4][colour 3]
 *             gauge  U  [T][Z][Y][X][mu 4][row 3][col 3]
 *   packed    the library's own device layouts (structure of arrays with the
 *             site index fastest). Their size is given by wd_spinor_bytes /
 *             wd_gauge_bytes; their contents are private to the library.
 *   memory    the caller allocates and frees every device buffer; the library
 *             never frees caller memory and allocates no device memory of
 *             its own in the apply calls.
 *   streams   every device call is asynchronous on the given stream (0 = the
 *             null stream) unless stated otherwise.
 *   errors    a negative wd_status. Argument errors are detected on the host
 *             before any launch; launch failures return WD_ERR_DEVICE;
 *             faults inside a kernel surface at the next synchronising call.
 *             wd_last_error() describes the last failure of this thread.
 *             Device pointers are checked with the HIP runtime: a host
 *             pointer, a pointer on another device, or a buffer whose HIP
 *             allocation ends before the bytes the call needs is rejected
 *             with WD_ERR_INVALID_ARG. (A sub-allocation of a caching
 *             allocator, e.g. a torch tensor, is checked against the segment
 *             that holds it; sizing it is the caller's job.) No C++
 *             exception crosses this interface.
 */
#ifndef WILSON_H
#define WILSON_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define WD_ABI_VERSION 4

#if defined(__GNUC__)
#define WD_API __attribute__((visibility("default")))
#else
#define WD_API
#endif

typedef enum wd_status {
  WD_OK = 0,
  WD_PENDING = 1,
  WD_ERR_INVALID_ARG = -1,
  WD_ERR_SHAPE = -2,
  WD_ERR_UNSUPPORTED = -3,
  WD_ERR_NOMEM = -4,
  WD_ERR_DEVICE = -5,
  WD_ERR_NOT_CONVERGED = -6,
  WD_ERR_NUMERIC = -7,
  WD_ERR_UNKNOWN_TICKET = -8,
  WD_ERR_CANCELLED = -9,
  WD_ERR_INTERNAL = -10
} wd_status;

/* Storage and arithmetic precision of a packed field.
 * WD_FP64: binary64 storage and arithmetic. WD_FP32: binary32 storage and
 * arithmetic. WD_FP16: binary16 storage, binary32 arithmetic; a spinor site is
 * stored as its 24 reals (rounded to binary32) divided by their largest
 * modulus, which is kept per site as a binary32 scale (52 bytes per site);
 * links are stored unscaled (entries of an SU(3) matrix are at most 1 in
 * modulus), each binary64 entry rounded once to binary16. Every rounding is
 * to nearest even. The paper keeps FP16 for compressing network data
 * (Sec. V-B); here it is a storage format that halves the bytes of FP32. */
typedef enum wd_prec { WD_FP64 = 0, WD_FP32 = 1, WD_FP16 = 2 } wd_prec;

/* flags of dslash_apply / dslash_apply_multi */
#define WD_FLAG_GAMMA5 1 /* return gamma5 D psi (the Hermitian Q = gamma5 D) */

typedef struct wd_gauge wd_gauge; /* opaque handle, owned by the library */

/* Version of this interface (WD_ABI_VERSION of the built library). */
WD_API int wd_abi_version(void);

/* Text of the last error on the calling thread; empty if none. The pointer
 * stays valid until the next call into the library on this thread. */
WD_API const char* wd_last_error(void);

/* Bytes of a packed spinor buffer holding nrhs fields of precision prec on a
 * lattice of extents dims (Sec. II-A: 12 complex numbers per site). Returns 0
 * for invalid arguments (bad dims, nrhs < 0, unknown precision). */
WD_API size_t wd_spinor_bytes(const int32_t dims[4], int32_t prec, int32_t nrhs);

/* Bytes of a packed gauge buffer (Sec. II-A: one SU(3) matrix per site and
 * direction). compress12 != 0 stores only the first two rows of each link
 * (12 reals); the third row is rebuilt as conj(row0 x row1), exact for SU(3).
 * Returns 0 for invalid arguments. */
WD_API size_t wd_gauge_bytes(const int32_t dims[4], int32_t prec, int32_t compress12);

/* Packs a canonical complex128 gauge field U_canon_dev into dst_dev (at least
 * wd_gauge_bytes(dims, prec, compress12) bytes, caller-owned, must outlive the
 * handle) and returns a handle in *out. The pack is enqueued on stream; the
 * handle may be used at once on the same stream. The canonical buffer is not
 * kept. With compress12 the input links must be SU(3) (unitary, det 1) for
 * the third row to be rebuilt exactly. Precisions: WD_FP64, WD_FP32, WD_FP16.
 * Errors: WD_ERR_INVALID_ARG (pointers, out == NULL, unknown precision),
 * WD_ERR_SHAPE (dims), WD_ERR_DEVICE (launch). */
WD_API int wd_gauge_import(const int32_t dims[4], const void* U_canon_dev, int32_t prec,
                    int32_t compress12, void* dst_dev, size_t dst_bytes,
                    hipStream_t stream, wd_gauge** out);

/* Releases a handle (host memory only; never frees dst_dev). NULL is a no-op.
 * The caller must not release a handle still used by enqueued work. */
WD_API int wd_gauge_release(wd_gauge* g);

/* Packs nrhs canonical complex128 spinor fields (canon_dev, layout above) into
 * dst_dev (wd_spinor_bytes(dims of g, prec, nrhs) bytes) in precision prec,
 * which must equal the precision of g. Enqueued on stream. */
WD_API int wd_spinor_import(const wd_gauge* g, const void* canon_dev, int32_t prec, int32_t nrhs,
                     void* dst_dev, hipStream_t stream);

/* Inverse of wd_spinor_import: unpacks nrhs packed fields src_dev into
 * canonical complex128 canon_dev. Enqueued on stream. */
WD_API int wd_spinor_export(const wd_gauge* g, const void* src_dev, int32_t prec, int32_t nrhs,
                     void* canon_dev, hipStream_t stream);

/* out = D(mass) in (eq. (1) of Sec. II-A in the (4+m) - H/2 normalisation,
 * see the top of this file), or gamma5 D(mass) in when flags has
 * WD_FLAG_GAMMA5. in_dev and out_dev are packed spinors of precision prec
 * (which must equal the precision of g) and must not overlap. mass = -4 gives
 * the pure hopping term -H/2. Asynchronous on stream.
 * Errors: WD_ERR_INVALID_ARG (NULL or overlapping buffers, precision mismatch,
 * unknown flags), WD_ERR_DEVICE (launch). */
WD_API int dslash_apply(const wd_gauge* g, double mass, const void* in_dev, void* out_dev,
                 int32_t prec, int32_t flags, hipStream_t stream);

/* out_k = D(masses_host[k]) in_k for k < nrhs (0..16; 0 is a no-op) in one
 * fused launch: the nrhs fields are consecutive packed spinors of precision
 * prec in in_dev and out_dev (wd_spinor_bytes(dims, prec, nrhs) bytes each;
 * eq. (1) of Sec. II-A per right-hand side, flags as for dslash_apply).
 * Each gauge link is fetched from HBM once per launch and served from L2 to
 * the other right-hand sides. Results equal nrhs separate dslash_apply calls
 * bit for bit. Asynchronous on stream.
 * Errors: WD_ERR_INVALID_ARG (buffers, masses, precision, flags),
 * WD_ERR_UNSUPPORTED (nrhs > 16), WD_ERR_DEVICE (launch). */
WD_API int dslash_apply_multi(const wd_gauge* g, const double* masses_host, int32_t nrhs,
                              const void* in_dev, void* out_dev, int32_t prec, int32_t flags,
                              hipStream_t stream);

/* ------------------------------------------------------------------------
 * Autotuner of the dslash launch (not from the paper: a search over launch
 * choices of the operator of eq. (1), Sec. II-A, on this device).
 *
 * Only choices that leave every site's arithmetic unchanged are searched: t
 * steps per workgroup, lane groups per workgroup, the run length of tiles
 * per XCD and right-hand sides per lane (1 or 2; with 2 a lane loads each
 * link once for both) of the t-marching kernel. A candidate is eligible only if its
 * output is bit-identical to the default choice's; the fastest eligible one
 * is kept in a process-wide cache keyed by (dims, prec, compress12, nrhs) and
 * used by every later dslash_apply / dslash_apply_multi / CG launch of that
 * key. The cache is empty at load time (defaults apply) and thread-safe.
 * ------------------------------------------------------------------------ */

typedef struct wd_tune_result {
  int32_t candidates;  /* launch choices timed (0: this lattice uses the one-site-per-lane kernel) */
  int32_t eligible;    /* of those, bit-identical to the default choice */
  int32_t tb, gw, group;  /* the choice kept: t steps and lane groups per workgroup, XCD run */
  int32_t rb;          /* ... and right-hand sides per lane */
  double default_us;   /* average time per launch of the default choice */
  double best_us;      /* ... and of the choice kept */
} wd_tune_result;

/* Times every eligible candidate for g's lattice with nrhs right-hand sides
 * (masses 0.1) in three interleaved rounds of reps launches each, and
 * registers the one with the fastest round (default_us and best_us are
 * fastest-round averages). in_dev
 * holds nrhs packed spinors of g's precision; out_dev and ref_dev are scratch
 * buffers of the same size, overwritten. Synchronous on stream; allocates a
 * few bytes of device memory for the comparison. Errors: WD_ERR_INVALID_ARG
 * (buffers, reps outside 1..1000), WD_ERR_UNSUPPORTED (nrhs), WD_ERR_DEVICE. */
WD_API int wd_tune_dslash(const wd_gauge* g, int32_t nrhs, const void* in_dev, void* out_dev,
                          void* ref_dev, int32_t reps, hipStream_t stream, wd_tune_result* result);

/* 1 and choice = {tb, gw, group, rb} if a choice is registered for the key,
 * 0 if not, negative for invalid arguments. */
WD_API int wd_tune_lookup(const int32_t dims[4], int32_t prec, int32_t compress12, int32_t nrhs,
                          int32_t choice[4]);

/* Forgets every registered choice. */
WD_API int wd_tune_reset(void);

/* Writes the registered choices to a text file (one line per key). */
WD_API int wd_tune_save(const char* path);

/* Adds the choices of a file written by wd_tune_save. Every line is checked
 * against its lattice (bounds, lanes, LDS); a file with any invalid line is
 * rejected whole with WD_ERR_INVALID_ARG and registers nothing. */
WD_API int wd_tune_load(const char* path);

/* ------------------------------------------------------------------------
 * Conjugate gradient on the normal equations D^dag D x = b.
 *
 * Sec. II-A of the paper names iterative solvers such as conjugate gradient
 * as where lattice QCD spends its time, dominated by the Dirac operator
 * applied to a quark field. D^dag D = Q^2 with the Hermitian Q = gamma5 D, so
 * every iteration applies dslash twice. With inner = WD_FP32 or WD_FP16 the
 * iterations run on fields of that precision (g_lo; FP16 storage keeps FP32
 * arithmetic) and accumulate the solution increments in FP32; whenever the
 * inner residual has dropped by delta since the last recompute or claims
 * convergence, the increments are added into the FP64 solution and the
 * residual is recomputed in FP64 (b - D^dag D x with g_hi: "reliable
 * updates"). Convergence is always decided on that FP64 true residual.
 * ------------------------------------------------------------------------ */

typedef struct wd_cg_params {
  double tol;          /* stop when |b - D^dag D x| <= tol |b| (FP64 true residual) */
  int32_t max_iter;    /* >= 1; iterations of the inner loop (each: two dslash) */
  int32_t inner;       /* WD_FP64 (plain CG), WD_FP32 or WD_FP16 (mixed precision) */
  double delta;        /* reliable-update threshold in (0, 1); used with mixed precision */
  int32_t check_every; /* >= 1; iterations between host checks of the residual */
  int32_t x0_given;    /* nonzero: start from the contents of x_dev, else x0 = 0 */
  int32_t use_graph;   /* nonzero: each run of check_every iterations is captured once as a
                          HIP graph (per set of unconverged right-hand sides) and replayed, on a
                          stream of the library's own ordered after `stream`; same results */
} wd_cg_params;

typedef struct wd_cg_stats {
  int32_t status;            /* WD_OK, WD_ERR_NOT_CONVERGED or WD_ERR_NUMERIC */
  int32_t iters;             /* inner iterations run */
  int32_t reliable_updates;  /* FP64 residual recomputations */
  int32_t reserved;
  double true_rel_residual;  /* |b - D^dag D x| / |b| at the last recompute */
  double seconds;            /* wall time of the whole call */
} wd_cg_stats;

/* Bytes of device workspace cg_solve_normal needs for nrhs right-hand sides
 * (1..16) on a lattice of extents dims with the given inner precision; 0 for
 * invalid arguments. */
WD_API size_t cg_workspace_bytes(const int32_t dims[4], int32_t nrhs, int32_t inner);

/* Solves D(m_k)^dag D(m_k) x_k = b_k for k < nrhs (1..16), each right-hand
 * side with its own mass masses_host[k]. b_dev and x_dev hold nrhs packed FP64
 * spinors of g_hi's lattice (wd_spinor_bytes(dims, WD_FP64, nrhs) bytes each;
 * x_dev is the output, and the start vector if params->x0_given). g_hi is an
 * FP64 gauge handle; g_lo a handle of the same lattice in the inner precision
 * when params->inner is WD_FP32 or WD_FP16 (ignored otherwise, may be NULL).
 * ws_dev:
 * cg_workspace_bytes(...) bytes of caller-owned device memory, not
 * overlapping b_dev or x_dev. stats_host: nrhs entries (may be NULL).
 * Synchronous: work is enqueued on stream and the call returns when every
 * right-hand side has converged, failed or used max_iter iterations. Every
 * check_every iterations the calling thread reads the scalars back and waits
 * for them by polling the stream (a busy wait; with use_graph, a blocking
 * wait); they land in a page-locked host buffer of 1,280 bytes that the
 * library takes from a pool of its own, one per call in progress, and keeps
 * for reuse until the process ends.
 * Returns WD_OK if all converged, else WD_ERR_NOT_CONVERGED or
 * WD_ERR_NUMERIC (per right-hand side detail in stats_host), or an argument
 * or device error. */
WD_API int cg_solve_normal(const wd_gauge* g_hi, const wd_gauge* g_lo, const double* masses_host,
                           int32_t nrhs, const void* b_dev, void* x_dev,
                           const wd_cg_params* params, wd_cg_stats* stats_host, void* ws_dev,
                           size_t ws_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Solving the Wilson system D x = b, and its even-odd (red-black) form.
 *
 * Sec. II-A of the paper says that iterative solvers such as conjugate
 * gradient, dominated by applications of the Dirac operator of eq. (1), take
 * most of a lattice QCD run; the system they solve is D x = b. On a lattice
 * whose four extents are all even, every hop of D joins sites of opposite
 * parity (x+y+z+t even or odd), so in the (even, odd) block order
 *   D = [[A, -H_eo/2], [-H_oe/2, A]],   A = 4 + m,
 * with H_pq the hopping term of eq. (1)'s operator from sites of parity q to
 * sites of parity p. Eliminating the even sites leaves the odd-site Schur
 * complement
 *   S = A - H_oe H_eo / (4 A),
 * and S x_o = b_o + H_oe b_e / (2A), x_e = (b_e + H_eo x_o / 2) / A solve
 * D x = b. S is gamma5-Hermitian and better conditioned than D.
 *
 * Even-odd fields: an even-odd gauge handle (wd_gauge_import_eo) stores the
 * links of the even sites, then those of the odd sites, each as a packed field
 * of V/2 sites; a half spinor field holds the sites of one parity (packed, V/2
 * sites per field, wd_spinor_eo_bytes). An even-odd handle also serves
 * wd_spinor_import / wd_spinor_export of full-lattice spinors (they use its
 * lattice only); dslash_apply, dslash_apply_multi, wd_tune_dslash and
 * cg_solve_normal need a full-lattice handle (WD_ERR_INVALID_ARG otherwise).
 * ------------------------------------------------------------------------ */

/* Bytes of an even-odd packed gauge buffer; 0 for invalid arguments or an odd
 * extent. */
WD_API size_t wd_gauge_eo_bytes(const int32_t dims[4], int32_t prec, int32_t compress12);

/* Bytes of nrhs half spinor fields (one parity, V/2 sites each); 0 for invalid
 * arguments or an odd extent. */
WD_API size_t wd_spinor_eo_bytes(const int32_t dims[4], int32_t prec, int32_t nrhs);

/* As wd_gauge_import, into the even-odd layout (dst_bytes >=
 * wd_gauge_eo_bytes). Every extent must be even (WD_ERR_SHAPE otherwise). */
WD_API int wd_gauge_import_eo(const int32_t dims[4], const void* U_canon_dev, int32_t prec,
                              int32_t compress12, void* dst_dev, size_t dst_bytes,
                              hipStream_t stream, wd_gauge** out);

/* Packs the sites of parity `parity` (0 even, 1 odd) of nrhs canonical
 * complex128 spinors into half spinor fields (wd_spinor_eo_bytes bytes),
 * precision prec = g's. Enqueued on stream. g: any handle of the lattice. */
WD_API int wd_spinor_import_eo(const wd_gauge* g, const void* canon_dev, int32_t prec, int32_t nrhs,
                               int32_t parity, void* dst_dev, hipStream_t stream);

/* Inverse of wd_spinor_import_eo: writes the half fields into the sites of
 * parity `parity` of nrhs canonical complex128 spinors and zero into the sites
 * of the other parity. Enqueued on stream. */
WD_API int wd_spinor_export_eo(const wd_gauge* g, const void* src_dev, int32_t prec, int32_t nrhs,
                               int32_t parity, void* canon_dev, hipStream_t stream);

/* out_k = S(masses_host[k]) in_k, or gamma5 S in_k with WD_FLAG_GAMMA5, for the
 * nrhs (0..16) odd half fields of in_dev; g an even-odd handle, prec = g's.
 * tmp_dev (nrhs half fields, overwritten) receives -H_eo in / 2 on the way.
 * in_dev, out_dev and tmp_dev must not overlap; masses must not be -4.
 * Asynchronous on stream. Errors as dslash_apply_multi. */
WD_API int dslash_apply_eo(const wd_gauge* g, const double* masses_host, int32_t nrhs,
                           const void* in_dev, void* out_dev, void* tmp_dev, int32_t prec,
                           int32_t flags, hipStream_t stream);

/* Bytes of device workspace cg_solve_wilson needs for nrhs (1..16)
 * right-hand sides, inner precision `inner`, and eo != 0 for even-odd gauge
 * handles; 0 for invalid arguments. */
WD_API size_t wilson_workspace_bytes(const int32_t dims[4], int32_t nrhs, int32_t inner, int32_t eo);

/* Solves D(m_k) x_k = b_k for k < nrhs, each with its own mass. b_dev and x_dev
 * hold nrhs full-lattice packed FP64 spinors (wd_spinor_bytes(dims, WD_FP64,
 * nrhs) bytes each; x_dev is the output, and the start vector if
 * params->x0_given). With full-lattice handles, CG solves the normal equations
 * D^dag D x = D^dag b (D^dag b = gamma5 D gamma5 b, formed on the device); with
 * even-odd handles (g_hi, and g_lo in the inner precision when params->inner
 * is WD_FP32 or WD_FP16), it solves S^dag S x_o = S^dag (b_o + H_oe b_e / (2A))
 * on the odd sites and rebuilds the even ones. Inner precision, reliable
 * updates, delta, check_every and use_graph as cg_solve_normal.
 * The call ends on the FP64 residual of the system itself: params->tol bounds
 * |b_k - D x_k| / |b_k|; CG first runs to tol on its own residual and resumes
 * with a tighter one where the system's residual is still above tol (at most
 * 6 runs, max_iter iterations in all). stats_host[k]: iterations and reliable
 * updates over all runs; true_rel_residual = |b_k - D x_k| / |b_k|.
 * ws_dev: wilson_workspace_bytes(...) bytes, not overlapping b_dev or x_dev.
 * Synchronous. Returns WD_OK if every right-hand side reached tol, else
 * WD_ERR_NOT_CONVERGED or WD_ERR_NUMERIC, or an argument or device error. */
WD_API int cg_solve_wilson(const wd_gauge* g_hi, const wd_gauge* g_lo, const double* masses_host,
                           int32_t nrhs, const void* b_dev, void* x_dev,
                           const wd_cg_params* params, wd_cg_stats* stats_host, void* ws_dev,
                           size_t ws_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * For callers that cannot allocate memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.
 * ------------------------------------------------------------------------ */

/* Size of the static device workspace of cg_solve_normal_noalloc (per GPU). */
#define WD_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* cg_solve_normal without a workspace argument. The workspace
 * (cg_workspace_bytes(dims, nrhs, params->inner) bytes, at most
 * WD_NOALLOC_SCRATCH_BYTES: e.g. 16^4 with one right-hand side, 8^4 with up to
 * 16) is a static device array of the library, one per GPU, held from the
 * first call on that GPU until the process ends. The call allocates nothing:
 * no hipMalloc, hipFree, hipHostMalloc or allocating library routine (its
 * first call on a device only looks up that array's address), and the
 * scalars it reads back land in a static pageable host buffer (one per GPU;
 * the copy into it waits for the stream). Every call on one GPU shares that
 * GPU's array and buffer, which keep the last call's contents (a call
 * initialises what it reads): calls that overlap in time on the same GPU, from
 * several threads, race and must be serialised by the caller.
 * params->use_graph is not supported (graph instantiation allocates):
 * WD_ERR_UNSUPPORTED. A solve needing more workspace than the limit:
 * WD_ERR_NOMEM (wd_last_error() gives the bytes needed). Arguments, results
 * and other errors as cg_solve_normal; results are bit-identical to it. */
WD_API int cg_solve_normal_noalloc(const wd_gauge* g_hi, const wd_gauge* g_lo,
                                   const double* masses_host, int32_t nrhs, const void* b_dev,
                                   void* x_dev, const wd_cg_params* params,
                                   wd_cg_stats* stats_host, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Request server: continuous batching of CG solves (cg_solve_normal's
 * algorithm) on gauge fields kept resident in a caller-given arena.
 *
 * A scheduler thread groups the right-hand sides of requests on the same
 * gauge field into slots that iterate together (one fused multi-right-hand-
 * side dslash per operator application). Requests join a group at chunk
 * boundaries (check_every iterations) as slots and arena memory free up, and
 * leave it when converged; groups of different lattices run on separate
 * streams and overlap on the device. A right-hand side gets bit-identical
 * results alone or in any mix. Requests wait (first fit in arrival order,
 * with a bound on how often one can be passed over) until a group of their
 * gauge field has free slots or the arena has room for a new group: one of
 * max_rhs_per_group slots, or, when that does not fit, one of just the
 * request's nrhs slots.
 * All server calls are thread-safe.
 * ------------------------------------------------------------------------ */

typedef struct wd_server wd_server; /* opaque */

typedef struct wd_server_cfg {
  void* arena_dev;            /* caller-owned device memory; the server owns it until destroyed */
  size_t arena_bytes;
  int32_t inner;              /* WD_FP32 or WD_FP16 (mixed precision), or WD_FP64 */
  int32_t check_every;        /* >= 1: CG iterations per chunk */
  double delta;               /* reliable-update threshold (mixed precision), in (0, 1) */
  int32_t max_rhs_per_group;  /* 1..16 slots per group; also the largest nrhs of a request */
  int32_t n_streams;          /* 1..16 streams the groups are spread over */
  int32_t evict_idle_gauges;  /* nonzero: wd_server_add_gauge evicts idle gauge fields (least
                                 recently used first) when the arena has no room */
} wd_server_cfg;

typedef struct wd_request {
  uint64_t gauge_id;    /* from wd_server_add_gauge */
  int32_t nrhs;         /* 1..max_rhs_per_group */
  int32_t max_iter;     /* >= 1 */
  double tol;           /* > 0: |b - D^dag D x| <= tol |b| per right-hand side */
  double masses[16];    /* masses[k] for k < nrhs */
  const void* b_dev;    /* nrhs packed FP64 spinors of the gauge field's lattice */
  void* x_dev;          /* nrhs packed FP64 spinors, written when the request completes */
} wd_request;

typedef struct wd_result {
  int32_t status;                       /* WD_PENDING, WD_OK, WD_ERR_NOT_CONVERGED, WD_ERR_NUMERIC, WD_ERR_CANCELLED */
  int32_t nrhs;
  double t_submit, t_start, t_done;     /* seconds since the server was created (-1: not yet) */
  wd_cg_stats stats[16];                /* per right-hand side; seconds = time since admission */
} wd_result;

typedef struct wd_server_state {
  size_t arena_in_use;   /* bytes of the arena allocated now */
  size_t arena_peak;     /* most bytes allocated at once so far */
  int32_t unfinished;    /* submitted requests not yet complete */
  int32_t gauges;        /* registered gauge fields */
  int32_t evictions;     /* gauge fields evicted to make room so far */
  int32_t reserved;
} wd_server_state;

/* Creates a server on the current device with its scheduler thread. The
 * arena must stay valid until wd_server_destroy returns. */
WD_API int wd_server_create(const wd_server_cfg* cfg, wd_server** out);

/* Packs the canonical complex128 gauge field U_canon_dev (FP64, plus a copy in
 * the inner precision for mixed precision) into the arena and returns its id;
 * U_canon_dev is not kept. Synchronous. If the arena has no room and
 * cfg.evict_idle_gauges is set, idle gauge fields (no request queued or
 * running on them) are evicted, least recently used (registered or named by
 * a request) first, until it fits; the id of an evicted field becomes unknown
 * (cg_submit returns WD_ERR_INVALID_ARG; register it again). WD_ERR_NOMEM if
 * the field cannot fit. */
WD_API int wd_server_add_gauge(wd_server* s, const int32_t dims[4], const void* U_canon_dev,
                               uint64_t* gauge_id);

/* The gauge field takes no new requests; its memory returns to the arena
 * once its queued and running requests are done. */
WD_API int wd_server_remove_gauge(wd_server* s, uint64_t gauge_id);

/* Queues a solve and returns at once with a ticket. b_dev and x_dev are
 * caller-owned and must stay valid until cg_poll reports a final status
 * (b_dev is copied into the arena when the request is admitted).
 * WD_ERR_NOMEM if a group of the request's nrhs slots cannot fit in the arena
 * beside the registered gauge fields. */
WD_API int cg_submit(wd_server* s, const wd_request* req, uint64_t* ticket);

/* WD_PENDING while the request is queued or running (out, if non-NULL, gets
 * the times so far); otherwise its final status, once: the ticket is then
 * forgotten (a later poll returns WD_ERR_UNKNOWN_TICKET). */
WD_API int cg_poll(wd_server* s, uint64_t ticket, wd_result* out);

/* Arena use and queue state (for footprint checks and monitoring). */
WD_API int wd_server_info(wd_server* s, wd_server_state* out);

/* Cancels queued and running requests (WD_ERR_CANCELLED, x not written),
 * waits for the device work in flight, joins the scheduler and frees the
 * server (not the arena). NULL is a no-op. */
WD_API int wd_server_destroy(wd_server* s);

#ifdef __cplusplus
} /* extern "C" */
#endif

#endif /* WILSON_H */

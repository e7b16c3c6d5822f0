/*
 * shtn -- Gauss-Legendre spherical harmonic transform for AMD MI355X (gfx950).
 *
 * Method: N. Schaeffer, "Efficient Spherical Harmonic Transforms aimed at
 * pseudo-spectral numerical simulations", arXiv 1202.6522.  Section numbers
 * below refer to that paper.
 *
 * Contents: plans (Gauss grid, recurrence tables, lane starts); the four
 * scalar transforms (synthesis, analysis and their adjoints) with the
 * Legendre stage recomputing P_n^m on the fly (Sec. 3.2) or reading a stored
 * table (Sec. 3.1), chosen per pass type by runtime tuning (Sec. 3.2); vector
 * (spheroidal / toroidal) transforms and their adjoints; batches of fields
 * of different truncations with graph capture and an autotuner; profiling.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  Truncation: degree n <= lmax, order 0 <= m <= min(n, mmax).
 *  Spectral arrays: complex FP64, interleaved (re, im) -- the memory layout of
 *    torch.complex128 / double _Complex -- in m-major triangular order
 *      idx(n, m) = m (2 lmax + 1 - m) / 2 + n,
 *    nlm = (mmax+1)(lmax+1) - mmax(mmax+1)/2 coefficients per field; fields are
 *    contiguous with stride nlm.  Only m >= 0 is stored: the fields are real,
 *    so f_n^{-m} = conj(f_n^m) (Sec. 3.1, Hermitian symmetry).  Im Q_n^0 is
 *    ignored on input and returned as 0.
 *  Grids: FP64 [nfields][nlat][nphi], row i = colatitude theta_i increasing
 *    (Gauss node x_i = cos theta_i decreasing, north to south), column
 *    k = longitude phi_k = 2 pi k / nphi.
 *  P_n^m: orthonormal associated Legendre functions with the (-1)^m
 *    Condon-Shortley factor of the definition in Sec. 2.1.
 *
 *  Pointers: every data pointer (Q, grid, work, device plan buffer) is a
 *    device pointer owned by the caller; arrays are contiguous.  `stream` is a
 *    hipStream_t passed as void* (NULL = the default stream).  The library
 *    allocates no device memory: tables and scratch live in caller buffers.
 *    Inputs are never modified.  A buffer a call writes (an output, the
 *    workspace) must share no byte with any other buffer of the call: its
 *    inputs, its other outputs, the plan's device and stored-P buffers, a
 *    batch's device buffer.  Buffers a call only reads may overlap.  Calls
 *    check this over the byte ranges their arguments define (nfields fields,
 *    the workspace size) and return SHTN_EINVAL, before any launch, when
 *    two ranges overlap; buffers that only touch are accepted.
 *  Errors: entry points return SHTN_OK (0) or a negative code below;
 *    shtn_last_error_detail() gives a thread-local message.  Transform calls
 *    are asynchronous on `stream`: a device fault surfaces at the caller's
 *    next synchronisation.  No C++ exception crosses this interface.
 */
#ifndef SHTN_H
#define SHTN_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SHTN_OK 0
#define SHTN_EINVAL (-1)       /* invalid argument (bad size, null pointer, short workspace) */
#define SHTN_EUNSUPPORTED (-2) /* valid but not implemented (e.g. nphi not a power of two)   */
#define SHTN_ESTATE (-3)       /* plan not uploaded to the device yet                         */
#define SHTN_EHIP (-4)         /* the HIP runtime reported an error                           */
#define SHTN_ENOMEM (-5)       /* host allocation failed                                      */

/* Fields per call: 1 .. SHTN_MAX_FIELDS for the scalar transforms (one
 * launch row per field), 1 .. SHTN_MAX_VEC_FIELDS for the vector transforms
 * (four scalar fields each); more give SHTN_EINVAL: split the call.
 * Batches have no such limit. */
#define SHTN_MAX_FIELDS 65535
#define SHTN_MAX_VEC_FIELDS 16383

typedef struct shtn_plan_s* shtn_plan_t;

/* Builds a transform plan on the host (no device call).
 * lmax >= 0, 0 <= mmax <= lmax, nlat >= 1 Gauss nodes (nlat >= lmax+1 makes
 * the analysis exact, Sec. 2.3), nphi equispaced longitudes with nphi > 2 mmax
 * and nphi a power of two.  Computes the Gauss nodes and weights (Sec. 2.3,
 * eq. gauss), the recurrence tables of Sec. 3.2 (eq. rec) in the rescaled form
 * used by the kernels, and -- by following every (order, latitude) recurrence
 * from P_m^m in a scaled-exponent form, the underflow guard of Sec. 3.5 run
 * at plan time -- the step at which each latitude's |P_n^m| first reaches
 * 2^-200 together with the recurrence state there.  The kernels start each
 * latitude at that step (before it every term is below 2^-200 and is dropped:
 * the polar optimisation of Sec. 3.1) and skip the steps in which no latitude
 * of a wave has started.  Also the restart states that split long orders into
 * balanced work units, the FFT twiddles and the work-unit lists.  Returns
 * NULL on error (see shtn_last_error_detail). */
shtn_plan_t shtn_plan(int lmax, int mmax, int nlat, int nphi);
void shtn_plan_destroy(shtn_plan_t plan); /* NULL is ignored */

/* Size in bytes of the device buffer that holds the plan's tables. */
size_t shtn_plan_device_bytes(shtn_plan_t plan);

/* Copies the plan's tables into the caller's device buffer `dev_buf`
 * (>= shtn_plan_device_bytes, 256-byte aligned) and synchronises `stream`.
 * The buffer must outlive every transform call with this plan. */
int shtn_plan_upload(shtn_plan_t plan, void* dev_buf, void* stream);

/* Device workspace bytes needed by a transform of `nfields` fields (the
 * longitude-Fourier coefficients F_m(theta_i) and the rescaled spectrum). */
size_t shtn_work_bytes(shtn_plan_t plan, int nfields);

/* Synthesis (Sec. 2.2): grid = S Q.
 * f(theta_i, phi_k) = Re F_0(theta_i) + 2 Re sum_{m=1}^{mmax} F_m(theta_i) e^{i m phi_k},
 * F_m(theta) = sum_{n=m}^{lmax} Q_n^m P_n^m(cos theta) (eq. synth_direct),
 * with P_n^m generated on the fly by the recurrence (Sec. 3.2) and the
 * equatorial mirror symmetry folded in (Sec. 3.1).
 * Q: nfields x nlm complex; grid: nfields x nlat x nphi. */
int shtn_synth(shtn_plan_t plan, const double* Q, double* grid, int nfields, void* work,
               void* stream);

/* Analysis (Sec. 2.3): Q = A grid.
 * F_m(theta_i) = (2 pi / nphi) sum_k f(theta_i, phi_k) e^{-i m phi_k},
 * Q_n^m = sum_i w_i P_n^m(x_i) F_m(theta_i) (eq. gauss).  Im Q_n^0 = 0. */
int shtn_analys(shtn_plan_t plan, const double* grid, double* Q, int nfields, void* work,
                void* stream);

/* Adjoint of the synthesis (the transpose of the real-linear map
 * (Re Q, Im Q) -> grid), returned as d + i e with d, e the Re and Im parts:
 * (S^T g)_n^m = c_m sum_i P_n^m(x_i) sum_k g_ik e^{-i m phi_k},
 * c_0 = 1, c_m = 2 (m >= 1).  With g = dL/dgrid this is the gradient of L with
 * respect to Q in PyTorch's complex convention (dL/dRe Q + i dL/dIm Q). */
int shtn_synth_adj(shtn_plan_t plan, const double* grid, double* Q, int nfields, void* work,
                   void* stream);

/* Adjoint of the analysis (transpose of grid -> (Re Q, Im Q)):
 * (A^T h)_ik = (2 pi / nphi) w_i [Re H_0(theta_i) + sum_{m>=1} Re(H_m(theta_i) e^{i m phi_k})],
 * H_m(theta) = sum_n h_n^m P_n^m(cos theta).  Im h_n^0 is ignored. */
int shtn_analys_adj(shtn_plan_t plan, const double* Q, double* grid, int nfields, void* work,
                    void* stream);

/* Plan queries (host only). */
long shtn_nlm(shtn_plan_t plan);
long shtn_lm_index(shtn_plan_t plan, int n, int m); /* -1 if (n, m) is outside the truncation */
/* Copies the nlat Gauss nodes x_i (decreasing) and weights w_i to host arrays. */
int shtn_get_grid(shtn_plan_t plan, double* x_host, double* w_host);
/* Algorithmic FP64 operations of one Legendre pass over one field:
 * 8 per (n, m, latitude pair) -- the recurrence step (3 multiplications and
 * one addition, Sec. 3.2) plus the complex multiply-accumulate. */
double shtn_legendre_flops(shtn_plan_t plan);

/* Copies a host-side plan table for inspection (tests, tools).
 * which: 0 x per pair, 1 sin(theta) per pair, 2 weight per pair (the middle
 * node of an odd grid carries half its weight), 3 beta (nlm), 4 gamma (nlm),
 * 5 P_m^m start mantissa ((mmax+1) x npair), 6 its scaled exponent k (int32,
 * same shape; value = mantissa 2^{-256 k}), 7 segment exponent shifts
 * (int32), 8 segment offsets per m (int32, mmax+2), 9 analysis restart
 * states (double, nrestart x npair x 2), 10 empty (kept for numbering),
 * 11 analysis units (int32 x 12 each), 12 synthesis units (int32 x 12 each),
 * 13 tiling (int32 x 9: synth_lp, analys_lp, fw, m_pairing, split, fft_rows,
 * analys_waves, start checkpoint spacing, polar threshold exponent),
 * 14 first latitude pair that
 * ever reaches the polar threshold, per m (int32), 15 start step of every
 * (order, pair) lane (int32, (mmax+1) x npair; lmax-m+1 = never), 16 the
 * recurrence state entering that step (double, (mmax+1) x npair x 2), 17 the
 * first start step of each block of 64 latitude pairs (int32, (mmax+1) x
 * ceil(npair/64)), 18 per (order, checkpoint k) two uint32 bit masks of
 * blocks 0..31: the blocks with a lane starting at step 8k, and those with
 * a lane started at or before it ((mmax+1) x ((lmax + 32)/8 + 2) x 2).
 * Returns the table size in bytes; copies only if dst != NULL and
 * bytes >= size.  Negative on error. */
long shtn_plan_table(shtn_plan_t plan, int which, void* dst, size_t bytes);

/* Tiling of the Legendre kernels (the runtime-tuning knob of Sec. 3.2):
 * synth_lp (1, 2, 4) latitude pairs per synthesis lane; analys_lp (1, 2, 4, 8)
 * pairs per analysis lane and analys_waves (1, 2, 4) waves per analysis unit,
 * which together must cover every latitude pair (64 analys_lp analys_waves >=
 * ceil(nlat/2); built combinations: waves 1 with lp 1-8, 2 with lp 2-8, 4
 * with lp 4 or 8); fields per synthesis wave fw (1, 2, 4; fw = 4 needs
 * synth_lp <= 2); the analysis takes min(fw, 2) fields per wave when
 * analys_lp <= 4 and analys_waves <= 2, else 1; m_pairing (synthesis: 0 one
 * workgroup per order, 1 orders m and mmax-m share a workgroup so that all
 * workgroups carry equal work); split (analysis n-range piece length, a
 * multiple of 32; 0 = automatic); fft_rows (latitude rows per FFT workgroup,
 * 0 = as many as fit).  Rebuilds the unit lists and restart tables:
 * re-upload afterwards.  Returns SHTN_EINVAL for unsupported values. */
int shtn_plan_set_tiling(shtn_plan_t plan, int synth_lp, int analys_lp, int analys_waves, int fw,
                         int m_pairing, int split, int fft_rows);

/* Polar threshold (Sec. 3.1, polar optimisation): every (order m, latitude
 * pair) lane enters the recurrence sums only from the first checkpoint
 * (multiple of 8 degrees) of the 8-degree block in which |P_n^m(x)| first
 * reaches 2^log2_threshold; earlier terms are dropped, and a latitude whose
 * |P_n^m| never reaches it for an order takes no part in that order.  The
 * default, -200, drops only terms below 1e-60 relative to the orthonormal
 * scale of P, so results match the plain definition to rounding.  Raising it
 * (say -40 to -20) skips more of the polar work at large lmax, at an error
 * of the order of 2^log2_threshold times the spectrum norm.  log2_threshold
 * must lie in [-1000, -1], else SHTN_EINVAL.  A threshold so low that some
 * stored lane start state would fall below the normal double range (a
 * denormal that has lost bits; about -900 at lmax 1023, -940 at lmax 255) is
 * refused with SHTN_EINVAL and the plan keeps its previous threshold.  Host
 * only: recomputes the lane starts, unit lists and restart tables; re-upload
 * afterwards (the plan is not uploaded until then, calls return
 * SHTN_ESTATE). */
int shtn_plan_set_polar(shtn_plan_t plan, int log2_threshold);

/* ---- synthesis without a workspace, for callers that cannot allocate ----
 *
 * For callers that cannot allocate device memory or provide a workspace:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same result as shtn_synth (bitwise: the same kernels), with the
 * workspace taken from a static device array of SHTN_NOALLOC_MAX_BYTES bytes
 * that every GPU the library runs on holds from the library's load until
 * the process ends.  Allocates nothing and calls no allocating routine.
 * SHTN_EINVAL when shtn_work_bytes(plan, nfields) exceeds
 * SHTN_NOALLOC_MAX_BYTES (one field at lmax 1023 fits, or five at lmax 511,
 * twenty at lmax 255); other errors as for shtn_synth.  All calls of one
 * process on one GPU share that GPU's array, which keeps the last call's
 * contents: calls that can overlap in time (on different streams, or from
 * host threads without ordering between them) race and give undefined
 * results; calls ordered on one stream do not.  Each process has its own
 * copy. */
#define SHTN_NOALLOC_MAX_BYTES ((size_t)32 << 20)
int shtn_synth_noalloc(shtn_plan_t plan, const double* Q, double* grid, int nfields, void* stream);

/* ---- vector (spheroidal / toroidal) transforms ----
 *
 * The paper names vector transforms but gives no formulas; the definition
 * used here is the usual one.  A tangent field on the unit sphere with
 * spheroidal potential S and toroidal potential T (spectra as for scalars,
 * same plan, Im of the m = 0 coefficients ignored) is
 *   V_theta = dS/dtheta - (1/sin theta) dT/dphi,
 *   V_phi   = (1/sin theta) dS/dphi + dT/dtheta,
 * on the plan's grid ([field][nlat][nphi] float64 per component).  The
 * analysis is the projection on the basis fields of each (n, m), divided by
 * their squared norm n(n+1): it inverts the synthesis for band-limited
 * fields (nlat >= lmax + 1); degree 0 comes out 0 and Im of m = 0 as 0.
 * Internally four scalar Legendre passes of modified spectra (or of
 * weighted longitude coefficients) with the plan's algorithm, tiling and
 * polar threshold, through sin(theta) dP_n^m/dtheta = n x P_n^m -
 * c_n P_{n-1}^m.  work: shtn_vec_work_bytes(plan, nfields) bytes of device
 * memory, 256-byte aligned.  Errors as for shtn_synth; the two outputs may
 * overlap no other buffer of the call (S and T may be one buffer, as may
 * Vtheta and Vphi on input). */
size_t shtn_vec_work_bytes(shtn_plan_t plan, int nfields);
int shtn_vec_synth(shtn_plan_t plan, const double* S, const double* T, double* Vtheta, double* Vphi, int nfields,
                   void* work, void* stream);
int shtn_vec_analys(shtn_plan_t plan, const double* Vtheta, const double* Vphi, double* S, double* T, int nfields,
                    void* work, void* stream);
/* Adjoints (transposes) of the two vector maps, for gradients: the adjoint of
 * the synthesis takes grids to spectra, that of the analysis spectra to
 * grids, with the scalar adjoints' conventions (gradient dRe + i dIm; degree
 * 0 and Im of order 0 carry nothing).  Same workspace and errors. */
int shtn_vec_synth_adj(shtn_plan_t plan, const double* Vtheta, const double* Vphi, double* S, double* T,
                       int nfields, void* work, void* stream);
int shtn_vec_analys_adj(shtn_plan_t plan, const double* S, const double* T, double* Vtheta, double* Vphi,
                        int nfields, void* work, void* stream);

/* ---- stored-P Legendre stage (Sec. 3.1, precomputed P_n^m) ----
 *
 * The second algorithm of the paper: P_n^m(x_i) stored for every order,
 * degree and northern latitude pair, read instead of recomputed.  With
 * several fields of one shape the Legendre stage is then a dense contraction
 * per order (pairs x degrees by degrees x (field, re/im)), run here on the
 * FP64 matrix cores; it trades the recurrence for reading the table
 * (8 ceil(nlat/2) nlm bytes plus padding: 0.29 GB at lmax 511, 2.2 GB at
 * lmax 1023), so it pays off with many fields per call.  Results agree with
 * the on-the-fly kernels to rounding: the table holds the same recurrence
 * values, and 0 where the polar threshold drops a term. */
#define SHTN_ALGO_ONTHEFLY 0       /* both passes recompute P (default)          */
#define SHTN_ALGO_STORED 1         /* both passes read the table                 */
#define SHTN_ALGO_STORED_SYNTH 2   /* synthesis-type passes (synthesis, adjoint  */
                                   /* of the analysis) read it, the others not   */
#define SHTN_ALGO_STORED_ANALYS 3  /* analysis-type passes (analysis, adjoint of */
                                   /* the synthesis) read it, the others not     */
/* Bytes of device memory the plan's table needs; negative on error. */
long shtn_ptable_bytes(shtn_plan_t plan);
/* Builds the table into dev_buf (device memory owned by the caller, 256-byte
 * aligned, at least shtn_ptable_bytes; it must stay allocated while the plan
 * uses it) from the uploaded plan, on `stream`, and waits for it.  The plan
 * records the buffer.  SHTN_ESTATE if the plan is not uploaded, SHTN_EINVAL
 * for a null, misaligned or short buffer.  A later shtn_plan_set_polar makes
 * the table stale: build it again. */
int shtn_ptable_build(shtn_plan_t plan, void* dev_buf, size_t bytes, void* stream);
/* Forgets the table (the caller may then free it) and selects the on-the-fly
 * algorithm. */
int shtn_ptable_release(shtn_plan_t plan);
/* Work decomposition of the stored-P kernels (one wave each): synthesis
 * synth_rt (1, 2, 4) tiles of 16 latitude pairs x synth_ct (1, 2) tiles of 8
 * fields; analysis analys_jt (1, 2, 4) tiles of 16 degrees of each parity x
 * analys_ct (1, 2) tiles of 8 fields.  Default 4, 2, 4, 2.  A call of at most 8
 * fields runs with one field tile whatever the setting.  SHTN_EINVAL for
 * other values.  Takes effect at the next call. */
int shtn_ptable_set_tiling(shtn_plan_t plan, int synth_rt, int synth_ct, int analys_jt, int analys_ct);
/* tiling4 = {synth_rt, synth_ct, analys_jt, analys_ct}. */
int shtn_ptable_get_tiling(shtn_plan_t plan, int* tiling4);
/* Selects the Legendre algorithm of the four transforms, one of SHTN_ALGO_*
 * (anything but SHTN_ALGO_ONTHEFLY needs a current table, else SHTN_ESTATE).
 * The FFT stages are the same for all. */
int shtn_plan_set_algorithm(shtn_plan_t plan, int algo);
/* The selected algorithm, or a negative error code. */
int shtn_plan_get_algorithm(shtn_plan_t plan);
/* Runtime tuning (Sec. 3.2): times `reps` synthesis calls (Q -> grid) and
 * `reps` analysis calls (grid -> Qout) of nfields fields with each algorithm
 * (the stored one only if the table is current), and selects for each pass
 * type the faster (the adjoints follow the pass they share kernels with).
 * us4 (may be NULL) receives the mean times in microseconds: synthesis
 * on-the-fly, synthesis stored, analysis on-the-fly, analysis stored (-1
 * when not timed).  Q, grid and Qout are device buffers of nfields fields;
 * Qout, like grid, may overlap no other buffer of the call.  Blocks until
 * done. */
int shtn_plan_tune_algorithm(shtn_plan_t plan, const double* Q, double* grid, double* Qout, int nfields,
                             void* work, void* stream, int reps, float* us4);

/* Measures the FP64 vector FMA rate (TFLOP/s, 2 flops per FMA) that the
 * current device sustains with four waves per SIMD on independent chains
 * with a scalar operand, the form of the Legendre kernels' inner loops: a
 * reference for their achieved FLOP/s next to the published peak.  Not part
 * of any transform.  Runs a few probe launches on `stream` (a hipStream_t)
 * and synchronises it.  Returns a negative value on a HIP error. */
double shtn_fp64_probe_tflops(void* stream);

/* ---- batches of fields with different truncations (one launch per stage) ----
 *
 * Many independent fields, each with its own truncation and grid, transformed
 * together: every stage of the transform is one kernel launch over all the
 * fields (the Legendre analysis one launch per class of latitude-pair count,
 * or a single one, see shtn_batch_set_tiling).  Same mathematics as
 * shtn_synth / shtn_analys applied field by field (Sec. 2 of the paper);
 * synthesis results are bitwise equal to the per-field calls at the same
 * synth_lp, analysis results agree to rounding.  The batching, graph capture
 * and tiling autotuner are this library's, not the paper's (its runtime
 * tuning of Sec. 3.2 picks among code variants per size; here the tuner picks
 * the work decomposition of the whole batch). */
typedef struct shtn_batch_s* shtn_batch_t;

/* A batch of nfields fields; field f is transformed with plans[f] (plans may
 * repeat).  The plans must stay alive and uploaded while the batch is used.
 * The batch copies each plan's device descriptor at its upload and builds its
 * unit tables from the plans' lane starts: after any change to a plan
 * (shtn_plan_upload, shtn_plan_set_tiling, shtn_plan_set_polar,
 * shtn_ptable_build or shtn_ptable_release) batch calls and replays return
 * SHTN_ESTATE until shtn_batch_upload, which rebuilds the tables.  Host only;
 * NULL on error (shtn_last_error_detail).  Packed buffers hold the fields
 * back to back in field order: spectra at q_off[f] doubles (2 per
 * coefficient, m-major as for a plan), grids at grid_off[f] doubles. */
shtn_batch_t shtn_batch(int nfields, const shtn_plan_t* plans);
void shtn_batch_destroy(shtn_batch_t batch);
/* q_off, grid_off: host arrays of nfields+1 entries, offsets in doubles (the
 * last entry is the packed total).  Either may be NULL. */
int shtn_batch_offsets(shtn_batch_t batch, size_t* q_off, size_t* grid_off);
/* Device bytes of the batch tables (largest over every tiling, so one buffer
 * serves the tuner) and of the workspace of a batched call. */
size_t shtn_batch_device_bytes(shtn_batch_t batch);
size_t shtn_batch_work_bytes(shtn_batch_t batch);
/* Copies the batch tables to dev_buf (caller-owned, 256-byte aligned, at least
 * shtn_batch_device_bytes) and waits for the copy.  Needed after creation,
 * after every shtn_batch_set_tiling and after a change to one of the plans
 * (the unit tables are rebuilt first; SHTN_ESTATE if they no longer fit the
 * size shtn_batch_device_bytes gave at creation); drops captured graphs. */
int shtn_batch_upload(shtn_batch_t batch, void* dev_buf, void* stream);
/* Batched synthesis / analysis of every field on `stream` (asynchronous).
 * Errors as for the plan calls; ESTATE if not uploaded. */
int shtn_batch_synth(shtn_batch_t batch, const double* Qpacked, double* gridpacked, void* work,
                     void* stream);
int shtn_batch_analys(shtn_batch_t batch, const double* gridpacked, double* Qpacked, void* work,
                      void* stream);
/* Tiling of the whole batch: synth_lp (1, 2, 4) latitude pairs per synthesis
 * lane; fw (1, 2, 4; 4 needs synth_lp <= 2) fields of the same plan per
 * synthesis wave (the analysis of a latitude-pair class takes min(fw, 2) or
 * 1, as for shtn_plan_set_tiling); m_pairing (0, 1):
 * synthesis units in longest-first order, or long and short units
 * alternating; analys_merge (0, 1): 0 launches the Legendre analysis once per
 * latitude-pair class (64, 128, 256, 512 pairs), 1 launches it once with the
 * largest class.  Re-upload afterwards. */
int shtn_batch_set_tiling(shtn_batch_t batch, int synth_lp, int fw, int m_pairing, int analys_merge);
/* tiling4 = {synth_lp, fw, m_pairing, analys_merge}. */
int shtn_batch_get_tiling(shtn_batch_t batch, int* tiling4);
/* Legendre algorithm of the batch: SHTN_ALGO_ONTHEFLY (default) or
 * SHTN_ALGO_STORED, with which the fields of every plan that has a current
 * stored-P table (shtn_ptable_build) run the stored kernels in both
 * directions (launched per plan, the fields addressed through the batch's
 * offset tables) and the other fields the on-the-fly kernels.  The plans'
 * tables must stay built while the batch uses them (calls return
 * SHTN_ESTATE otherwise).  Re-upload afterwards.  The tuner
 * (shtn_batch_tune) tries both when any plan has a table. */
int shtn_batch_set_algorithm(shtn_batch_t batch, int algo);
int shtn_batch_get_algorithm(shtn_batch_t batch);
/* Captures the launch sequence of one direction (which = 0 synthesis
 * in -> out, 1 analysis) into a hipGraph held by the batch, on a private
 * stream, for these exact buffers.  Replaying it (shtn_batch_replay) on any
 * stream runs the transform on those buffers.  The graph holds kernel nodes
 * only (no memset or copy nodes).  Uploading again drops the graphs; a
 * replay after a change to one of the plans returns SHTN_ESTATE. */
int shtn_batch_capture(shtn_batch_t batch, int which, const double* in, double* out, void* work);
int shtn_batch_replay(shtn_batch_t batch, int which, void* stream);
/* Autotuner: times a synthesis (Qpacked -> gridpacked) plus analysis
 * (gridpacked -> Qout) round trip of graph replays for every tiling
 * (synth_lp 1|2, fw 1|2|4, m_pairing 0|1, analys_merge 0|1, and both batch
 * algorithms when a plan has a stored-P table; reps replays each,
 * default 10 when reps < 1), keeps the fastest, re-uploads and leaves both
 * graphs captured for these buffers.  Blocks until done.  With cache_path
 * (may be NULL), a tiling stored there for the same list of field shapes and
 * the same GPU architecture is used without timing, and a new result is
 * appended; entries that do not parse or name a tiling outside the values
 * above are ignored (the candidates are timed).  *best_us (may be NULL)
 * receives the best round-trip time, or -1 when taken from the cache.  The
 * batch must be uploaded; Qout may overlap no other buffer of the call. */
int shtn_batch_tune(shtn_batch_t batch, const double* Qpacked, double* gridpacked, double* Qout,
                    void* work, void* stream, int reps, const char* cache_path, float* best_us);

/* ---- kernel timing for benchmarks ----
 * When enabled, every kernel launched by the library is bracketed by a pair of
 * HIP events recorded on the launch stream.  shtn_profile_read waits for the
 * recorded events and returns, for one kernel kind, the summed duration in
 * milliseconds and the number of launches since the last reset.  Kinds:
 * 0 spectrum rescale, 1 Legendre synthesis, 2 Legendre analysis,
 * 3 Fourier synthesis (c2r), 4 Fourier analysis (r2c).  Not for use under
 * stream capture.  shtn_profile_select restricts the timing to the kinds
 * whose bit is set in kind_mask (all kinds by default): every event pair
 * costs a few microseconds of GPU time between kernels. */
int shtn_profile_enable(int on);
int shtn_profile_select(unsigned kind_mask);
int shtn_profile_read(int kind, double* total_ms, long* launches);
void shtn_profile_reset(void);

/* Error reporting. */
const char* shtn_strerror(int code);
const char* shtn_last_error_detail(void);

#ifdef __cplusplus
}
#endif
#endif /* SHTN_H */

/*
 * tufrg.h -- C ABI of the MI355X truncated-unity fRG right-hand side.
 *
 * The library evaluates the right-hand side of the truncated-unity fRG flow
 * of multiband systems without SU(2) symmetry (Schober, Ehrlich, Reckling,
 * Honerkamp, arXiv:1710.08830) in the orbital/spin basis, and integrates it:
 *
 *   dP(s)/dLambda = VP(s) Lpp(s) VP(s)            (Sec. 3.1 matrix RGE for P,
 *   dC(u)/dLambda = 2 VC(u) Lph(u) VC(u)           orbital form of Sec. 4.2)
 *
 * with the projected vertices VP = P[V0] + P + P[V^C] + P[V^D] and
 * VC = C[V0] + C[V^P] + C + C[V^D] of Sec. 3.3, and D = -C with the last two
 * orbital indices exchanged (Sec. 3.2), so only P and C are stored.
 *
 * ---------------------------------------------------------------------------
 * Conventions
 *
 * Meshes.  Momentum transfers q run over the coarse mesh q = 2 pi (mx, my)/Lq,
 * linear index mx * Lq + my, Nq = Lq^2.  Loops average over the refined mesh
 * k = 2 pi (kx, ky) / Lf with Lf = n_ref * Lq (coarse point m is fine point
 * n_ref * m, so k +- q stays on the fine mesh), Nf = Lf^2.
 *
 * Form factors.  Plane waves f_R(k) = exp(-i k.R) (Sec. 2 and Sec. 3.3), labelled
 * by the bond vectors R of the list ff_R; ff_R[0] must be (0, 0), the list must
 * be closed under R -> -R, and |R_x|, |R_y| <= 2.
 *
 * Bundle layout.  With n_o spin-orbitals and n_ff form factors the bundle
 * dimension is B = n_ff * n_o^2, and a row or column index is
 * i = r * n_o^2 + a * n_o + b (form factor r, orbitals a, b).  The exchange
 * propagators are complex B x B matrices per coarse q:
 *     P[q][(R,a,b)][(R',c,d)] = P^{RR'}_{a b d c}(q)    rows n1 n2, columns n4 n3
 *     C[q][(R,a,b)][(R',c,d)] = C^{RR'}_{a d b c}(q)    rows n1 n3, columns n4 n2
 * so that the matrix RGE above is a plain product of B x B matrices, and the
 * hermiticity of the projections (Sec. 2, property 3) is matrix hermiticity.
 * Arrays are row-major [Nq][B][B] of tufrg_c64.
 *
 * Loops.  Lpp and Lph are the orbital loop matrices
 *   Lpp(s)[(R1,a,b),(R2,c,d)] = 1/Nf sum_k e^{-ik.(R1-R2)}
 *        sum_mn Pi_m(k)_ac Pi_n(s-k)_bd L-(e_m(k), e_n(s-k))
 *   Lph(u)[(R1,a,b),(R2,c,d)] = 1/Nf sum_k e^{-ik.(R1-R2)}
 *        sum_mn Pi_m(k)_ac Pi_n(k-u)_db L+(e_m(k), e_n(k-u))
 * with e_m = E_m - mu and Pi_m(k) = U_m U_m^dagger the band projectors of H(k)
 * (Sec. 4.1).  L-/+ = d/dLambda of the regulated bubbles F-/+ of Sec. 3.1:
 * the temperature flow (Lambda = T) or the Omega scheme at T = 0 (propagator
 * times w^2 / (w^2 + Omega^2)).
 *
 * Interaction.  V0 is the antisymmetric onsite initial vertex V0[n1][n2][n3][n4]
 * in the normalisation H_int = 1/2 sum V0_{1234} c+_1 c+_2 c_4 c_3 (the onsite
 * Hubbard vertex of Sec. 5 is U/2 (d13 d24 - d14 d23)).  Its projections fill
 * the (0,0) form-factor block only.
 *
 * ---------------------------------------------------------------------------
 * Ownership, execution, errors
 *
 * Model and setup arrays are host memory, read during tufrg_create only.
 * Every P, C, VP, VC, L, dP, dC argument is DEVICE memory allocated by the
 * caller (e.g. a torch tensor of dtype complex128); the library never frees
 * caller memory.  A host pointer is rejected with TUFRG_E_INVAL.  The context
 * owns its band data, tables and workspaces.
 *
 * All calls are enqueued on the stream given to tufrg_create and are
 * asynchronous, except these, which synchronise that stream: tufrg_create and
 * tufrg_destroy; tufrg_flow and tufrg_batch_flow, once per step, to read back
 * the stop test (a few bytes); tufrg_ff_apply (its W is a host array);
 * tufrg_timing and tufrg_timing_read; tufrg_sur_targets when max_abs is
 * requested; and the network calls that return host values or reshape their
 * buffers (tufrg_mlp_create, _destroy, _loss_grad, _train).
 * A context must be used by one host thread at a time.  No exception or abort
 * crosses the ABI: failures return a status, and tufrg_last_error() returns a
 * message (per context, or the calling thread's last create failure for NULL).
 * Divergence of a flow is a result (diverged = 1), not an error.
 */
#ifndef TUFRG_H
#define TUFRG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tufrg_ctx tufrg_ctx;

/* binary-compatible with C99 double _Complex and torch.complex128 */
typedef struct {
  double re, im;
} tufrg_c64;

typedef enum {
  TUFRG_OK = 0,
  TUFRG_E_INVAL = 1,       /* bad argument (null, host pointer, unsupported shape) */
  TUFRG_E_NOMEM = 2,       /* device allocation failed */
  TUFRG_E_HIP = 3,         /* a HIP runtime call failed */
  TUFRG_E_NONFINITE = 4,   /* NaN or Inf in the state during a flow */
  TUFRG_E_STEPSIZE = 5,    /* adaptive step size underflow */
  TUFRG_E_UNSUPPORTED = 6  /* valid request the library does not implement */
} tufrg_status;

/* Regulators (Sec. 3.1: the loops are the Lambda derivatives of regulated
 * bubbles).  TEMPERATURE: Lambda = T.  OMEGA: frequency cutoff
 * w^2 / (w^2 + Lambda^2) at T = 0.  SHELL: the paper's momentum-shell
 * regulator at a fixed temperature (tufrg_setup.temperature): each propagator
 * times chi_Lambda(e) = e^2 / (e^2 + Lambda^2), a smooth shell of width Lambda
 * around the Fermi surface (the paper leaves the shape open). */
typedef enum { TUFRG_CUT_TEMPERATURE = 0, TUFRG_CUT_OMEGA = 1, TUFRG_CUT_SHELL = 2 } tufrg_cutoff;

/* Single-particle basis of the exchange propagators.  ORBITAL: the loops of
 * Sec. 4.2 with the band projectors Pi_m(k) of H(k).  BAND: the eigenbasis of
 * H(k) (the form in which Sec. 3.1 writes the RGE): the loops see unit
 * projectors and depend on two band indices, L(e_l1(k'), e_l2(k)); the
 * projections and bundle products are unchanged.  A band-basis state depends
 * on the eigenvector gauge of the basis change that produced it; the bare
 * vertex is then given as a static P term (tufrg_set_initial_p, e.g.
 * U^H P[V0] U from tufrg_basis_matrix / tufrg_basis_apply) with V0 = 0 in the
 * model. */
typedef enum { TUFRG_BASIS_ORBITAL = 0, TUFRG_BASIS_BAND = 1 } tufrg_basis;

/* Arithmetic of the loops and bundle products; the state and its updates are
 * always FP64.  TUFRG_FP32 accumulates each loop k-chunk in FP32 and sums
 * chunks in FP64.  TUFRG_BF16X3 (six spin-orbitals only) runs the loop's k
 * contraction on the matrix cores, in the real basis of Hermitian matrices,
 * with BF16 split operands (v = hi + lo, three products per pair), FP32
 * accumulation along each kx row and an FP64 sum over rows; bundle products
 * with B > 64 also run on the matrix cores, each complex product as four real
 * ones of split operands with FP32 accumulation (the intermediate L V split
 * again); everything else as TUFRG_FP32. */
typedef enum { TUFRG_FP64 = 0, TUFRG_FP32 = 1, TUFRG_BF16X3 = 2 } tufrg_precision;

typedef enum { TUFRG_PP = 0, TUFRG_PH = 1 } tufrg_channel;

typedef struct {
  int32_t n_orb;           /* spin-orbitals n_o: 2 or 6; or 1: one orbital per site with spin-rotation
                              invariance, for the SU(2)-reduced calls (tufrg_su2_rhs, tufrg_su2_flow;
                              V0 is then the onsite coefficient v of d13 d24 - d14 d23) */
  int32_t n_hop;           /* hopping vectors */
  const int32_t *hop_R;    /* [n_hop][2] lattice vectors R */
  const tufrg_c64 *hop_t;  /* [n_hop][n_o][n_o]: H(k) = sum_R t(R) e^{i k.R}; t(-R) = t(R)^dagger */
  double mu;               /* chemical potential */
  const tufrg_c64 *V0;     /* [n_o]^4 antisymmetric onsite vertex, order n1 n2 n3 n4 */
} tufrg_model;

typedef struct {
  int32_t n_ff;            /* number of form factors */
  const int32_t *ff_R;     /* [n_ff][2], ff_R[0] = (0,0), closed under negation, |R_x|,|R_y| <= 2;
                              six spin-orbitals: every difference R1 - R2 inside the 5 x 5 box
                              |dx|, |dy| <= 2 or the diamond |dx| + |dy| <= 4 (else TUFRG_E_UNSUPPORTED) */
  int32_t Lq;              /* coarse mesh; must exceed 4 max|R| (no aliasing in R'' = R1 - R2) */
  int32_t n_ref;           /* refinement of the loop mesh, Lf = n_ref Lq <= 4096 */
  int32_t cutoff;          /* tufrg_cutoff */
  int32_t precision;       /* tufrg_precision */
  double temperature;      /* TUFRG_CUT_SHELL: the fixed temperature T > 0 of its bubbles; ignored otherwise */
  int32_t basis;           /* tufrg_basis: single-particle basis of the state (orbital by default) */
} tufrg_setup;

/* Builds meshes, tables and the band data (eigendecomposition of H(k) - mu on
 * the fine mesh, FP64, on the device).  stream: a hipStream_t or NULL. */
tufrg_status tufrg_create(const tufrg_model *model, const tufrg_setup *setup, void *stream, tufrg_ctx **out);
tufrg_status tufrg_destroy(tufrg_ctx *ctx);
const char *tufrg_last_error(const tufrg_ctx *ctx);

/* Sizes: B, Nq, Nf, and the number of distinct R1 - R2 differences. */
tufrg_status tufrg_dims(const tufrg_ctx *ctx, int32_t *B, int32_t *Nq, int32_t *Nf, int32_t *n_dR);

/* Band data (diagonalisation of H(k), Sec. 4.1, built by tufrg_create): e[m][k] = E_m(k) - mu
 * (ascending in m) and the projectors Pi[m][k][a][c] = U_am(k) conj(U_cm(k)),
 * k = kx * Lf + ky.  Device arrays of n_o * Nf doubles and n_o * Nf * n_o^2
 * tufrg_c64. */
tufrg_status tufrg_band_data(tufrg_ctx *ctx, double *e, tufrg_c64 *Pi);

/* Loop matrices of one channel at scale lambda for every coarse q:
 * L[q][B][B] in the bundle layout (see above).  deriv = 1: L-/+ = dF/dLambda
 * (the loops of the RGE); deriv = 0: the bubbles F-/+ themselves. */
tufrg_status tufrg_bubble(tufrg_ctx *ctx, int32_t channel, double lambda, int32_t deriv, tufrg_c64 *L);

/* Non-local part of the initial interaction (the paper's outlook: longer-ranged
 * bare interactions, whose projections fill form-factor blocks beyond (0,0)):
 * C0 [Nq][B][B] (device, the C bundle layout) is a static crossed
 * particle-hole term of the bare vertex.  From this call on every projection
 * uses C + C0 in place of C (and D + D0, D0 = -C0 with the last two indices
 * exchanged, Sec. 3.2), so 'VP = P[V0] + P + P[V^C] + P[V^D]' and 'VC' include
 * the projections of the non-local bare interaction while the flowing state C
 * starts from zero.  A density-density interaction (1/2) sum_{i,d} V_d n_i
 * n_{i+d} has C0^{00}(u)_{n1n2n3n4} = (1/2) sum_d V_d e^{-iu.d} d13 d24 in the
 * (0,0) form-factor block (the onsite d = 0 term is V0).  The library copies
 * C0 (stream-ordered); C0 = NULL removes it.  Errors: E_INVAL for a host
 * pointer, E_NOMEM when the two [Nq][B][B] buffers cannot be allocated. */
tufrg_status tufrg_set_initial_c(tufrg_ctx *ctx, const tufrg_c64 *C0);

/* Orbital <-> band basis (Sec. 4.1).  The basis change of a vertex with the
 * unitary U(k) that diagonalises H(k) turns, for the projected matrices, into
 * sandwiches with the form-factor averages
 *   U^{RR'}_{s1s2n1n2}(s) = 1/Nf sum_k f_R(k) f*_R'(k) U_{s1n1}(s-k) U_{s2n2}(k)   (pp)
 *   X^{RR'}_{s1s2n1n2}(u) = 1/Nf sum_k f_R(k) f*_R'(k) U_{s1n1}(k) U*_{s2n2}(k-u)  (ph)
 * (s orbital, n band indices, sums over the fine mesh).  In the bundle layout
 * they are the matrices
 *   M_pp[q][(R,a,b)][(R',c,d)] = U^{RR'}_{b a d c}(q),  M_ph[q][(R,a,b)][(R',c,d)] = X^{RR'}_{a b c d}(q),
 * and the laws of the paper read Pb = M_pp^H P M_pp, Cb = M_ph^H C M_ph per q
 * (converse: P = M_pp Pb M_pp^H, C = M_ph Cb M_ph^H; exact inverses only for a
 * complete form-factor set on an unrefined mesh).  The band-basis quantities
 * depend on the phases of the eigenvectors (and on the basis chosen inside
 * degenerate subspaces), so U is an input: U[k][a][n] = U_an(k), k = kx * Lf
 * + ky, Nf * n_o^2 tufrg_c64 on the device, unitary per k (not checked).
 * tufrg_basis_matrix writes M [Nq][B][B] (device) for channel TUFRG_PP (U
 * matrix) or TUFRG_PH (X matrix); every entry is a fixed-order FP64 k-sum.
 * Workspaces (a compact [2][Nq][n_dR][n_o^4] table and a row buffer of at
 * most 1 GiB) are allocated on the first call and kept with the context.
 * Errors: E_INVAL for an unknown channel or a host pointer, E_NOMEM when a
 * workspace cannot be allocated (retried on the next call). */
tufrg_status tufrg_basis_matrix(tufrg_ctx *ctx, int32_t channel, const tufrg_c64 *U, tufrg_c64 *M);

/* Y[q] = M[q]^H X[q] M[q] (to_orbital = 0: orbital -> band) or
 * Y[q] = M[q] X[q] M[q]^H (to_orbital = 1: band -> orbital), all [Nq][B][B]
 * on the device, FP64.  Y may be X; it must not overlap M.  A workspace of
 * Nq * B * B tufrg_c64 is allocated on the first call and kept.  Errors:
 * E_INVAL for a host pointer or Y overlapping M, E_NOMEM for the workspace. */
tufrg_status tufrg_basis_apply(tufrg_ctx *ctx, const tufrg_c64 *M, const tufrg_c64 *X, tufrg_c64 *Y,
                               int32_t to_orbital);

/* Point-group-symmetrised form factors.  The plane waves f_R(k) = e^{-ik.R}
 * of a form-factor set closed under C4v recombine into f~_i = sum_R W_iR f_R
 * (W unitary) that transform under its irreducible representations; a
 * propagator then changes by X~ = W X W^H in the form-factor index (orbital
 * indices untouched), the converse X = W^H X~ W.
 * tufrg_ff_symmetrize (host only, no context): W [n_ff][n_ff] (rows) and the
 * label of each row, 0 A1, 1 A2, 2 B1, 3 B2, 4 E x-like, 5 E y-like, for S
 * given as ff_R [n_ff][2].  Orbits in order of first appearance in S; inside
 * an orbit A1, then B1 (axis shells: cos kx - cos ky) or B2 (diagonal
 * shells), then the E pair (x-like: odd under x -> -x, even under y -> -y);
 * each row's first nonzero coefficient (in the order of S) real and positive.
 * W, irrep: host arrays owned by the caller.  Errors: E_INVAL when S is not a
 * union of C4v orbits (or has duplicates, or n_ff > 25), E_UNSUPPORTED for
 * orbits of eight vectors (such as (1, 2)).
 * tufrg_ff_apply: Y[q] = X~ (to_plane_waves = 0) or the converse (1) for
 * [Nq][B][B] device arrays in the bundle layout (P or C alike: the orbital
 * pairs are untouched); W host [n_ff][n_ff].  Synchronises the context's
 * stream.  A 25 x 25 device copy of W is allocated on the first call and
 * kept.  Errors: E_INVAL for a null or device W, host X/Y, overlapping X and
 * Y; E_NOMEM when the copy of W cannot be allocated. */
tufrg_status tufrg_ff_symmetrize(int32_t n_ff, const int32_t *ff_R, tufrg_c64 *W, int32_t *irrep);
tufrg_status tufrg_ff_apply(tufrg_ctx *ctx, const tufrg_c64 *W, const tufrg_c64 *X, tufrg_c64 *Y,
                            int32_t to_plane_waves);

/* Static particle-particle term of the bare vertex: P0 [Nq][B][B] (device,
 * the P bundle layout) is the P-channel expansion of (part of) the bare
 * vertex.  From this call on every projection uses P + P0 in place of P, so VP
 * includes P0 and VC its crossed particle-hole projection (Sec. 3.3).  An
 * onsite interaction is exactly its (0,0) block; the band-basis form of an
 * orbital interaction is U^H P[V0] U (Sec. 4.1), exact for a complete
 * form-factor set and its truncated expansion otherwise.  The library copies
 * P0 (stream-ordered); P0 = NULL removes it.  Errors: E_INVAL for a host
 * pointer, E_NOMEM when the two [Nq][B][B] buffers cannot be allocated. */
tufrg_status tufrg_set_initial_p(tufrg_ctx *ctx, const tufrg_c64 *P0);

/* Result of tufrg_autotune. */
typedef struct {
  int32_t tunable;        /* 0: this setup has no launch shape to tune (six spin-orbitals on
                             the vector units: one workgroup per q and channel) */
  int32_t from_cache;     /* 1: the shape came from the cache file; nothing was timed */
  int32_t loop_kx_chunks; /* two spin-orbitals: kx chunks of the loop kernel now in use */
  int32_t mfma_kx_rows;   /* six spin-orbitals, BF16X3: kx rows per work item now in use */
  int32_t n_candidates;   /* shapes timed (0 from the cache) */
  double loop_ms;         /* one evaluation of both loop channels with the chosen shape */
  double default_ms;      /* the same with the shape the context started with */
} tufrg_tune_result;

/* Launch-shape autotuner of the loop kernels (no passage: an implementation
 * choice).  Times one evaluation of both loop channels at scale lambda (HIP
 * events on the context's stream, one untimed evaluation first, then about
 * 50 ms of repeats) for each candidate shape and keeps the fastest in the
 * context: for two spin-orbitals the number of kx chunks of the loop kernel
 * (partial sums per chunk, the buffer grows if a candidate needs more), for
 * TUFRG_BF16X3 the kx rows per matrix-core work item.  The shape only
 * regroups the k sum: BF16X3 results are unchanged bit for bit, two-orbital
 * ones change by FP32 rounding of the chunk partials.  cache_path (may be
 * NULL) names a JSON file {"version": 1, "entries": {"<key>": {...}}} keyed
 * by GPU architecture, compute units and problem shape: an entry for this
 * shape is applied without timing; otherwise the result is added and the
 * file rewritten (through a temporary file and a rename).  Synchronous.  The
 * chosen shape stays until the context is destroyed or tuned again.  Errors:
 * E_INVAL for a null result, lambda <= 0, a cache file that exists but is not
 * a tuning cache (left untouched) or cannot be written; E_NOMEM, E_HIP as the
 * loops.  Call it outside flows and graph captures. */
tufrg_status tufrg_autotune(tufrg_ctx *ctx, double lambda, const char *cache_path, tufrg_tune_result *res);

/* Kramers-paired bands in the six-orbital loops (no passage: an
 * implementation choice that the sum over bands of the Sec. 3.1 loop
 * permits).  When the six bands are degenerate in pairs (0,1), (2,3), (4,5) at
 * every k of the fine mesh (time reversal with inversion symmetry; checked at
 * creation: splittings at most 1e-10 max(1, max |e|)), the loops sum each
 * degenerate pair first: three energies and three summed projectors (BF16X3:
 * also L_f even; half the matrix-core work per k; FP32 and FP64: half the
 * band sum and a quarter of the W build per k).  Exact for exactly degenerate
 * bands; the eigensolver's splittings (about 1e-14) change the loops far
 * below the rounding of FP32 and BF16X3 and within 1e-11 in FP64.
 * enable = 1 (the default) uses the pairs where they were found, 0 always
 * uses the six bands; *active (may be NULL) receives whether the pairs are in
 * use.  If the choice changed and the precomputed A operand of the loops
 * exists, it is rebuilt in this call (synchronous; E_NOMEM or E_HIP as the
 * loops).  Call it outside flows and graph captures.  Errors: E_INVAL for a
 * null context or enable not 0 or 1. */
tufrg_status tufrg_pair_bands(tufrg_ctx *ctx, int32_t enable, int32_t *active);

/* The third channel (Sec. 3.2): D_{n1n2n3n4} = -C_{n1n2n4n3}, which the
 * antisymmetry of the vertex fixes, so only P and C flow.  C and D are device
 * arrays [Nq][B][B] on the context's device; D is written in the layout of C,
 * D[q][(R,a,b)][(R',c,d)] = D^{RR'}_{a d b c}(q) = -C[q][(R,a,c)][(R',b,d)]
 * (exact, no arithmetic beyond the sign).  The caller owns both; they must not
 * overlap.  Asynchronous on the context's stream.  Errors: E_INVAL for a host
 * pointer or overlapping arrays, E_HIP for a failed launch. */
tufrg_status tufrg_channel_d(tufrg_ctx *ctx, const tufrg_c64 *C, tufrg_c64 *D);

/* Projected vertices VP, VC [Nq][B][B] of the state P, C [Nq][B][B] (Sec. 3.3). */
tufrg_status tufrg_project(tufrg_ctx *ctx, const tufrg_c64 *P, const tufrg_c64 *C, tufrg_c64 *VP,
                           tufrg_c64 *VC);

/* The projections of tufrg_project for callers that cannot allocate device
 * memory (code under HIP graph capture, serving loops, harnesses that forbid
 * hipMalloc): the same VP, VC, with the rho-space buffers (the transforms'
 * intermediate, the coefficients P(rho), C(rho) and the gathers) in a static device array of
 * 32 MiB that the library holds on each GPU until the process ends.  The call
 * allocates nothing; the context must have been created (its own allocation
 * happens there) with the same device current as now.  Limit: 3 * 4 * n_dR *
 * B^2 doubles must fit in 32 MiB (B <= 64 with n_dR <= 41; the six-orbital
 * B = 468 setups are rejected with TUFRG_E_UNSUPPORTED).  Every buffer is
 * written before it is read, so nothing carries over between calls, but all
 * calls on one GPU share the array: calls that overlap in time on one GPU
 * (several streams or host threads) race and must be serialised by the
 * caller.  Errors: E_INVAL for a host pointer or another current device,
 * E_UNSUPPORTED for a setup beyond the limit. */
tufrg_status tufrg_project_static(tufrg_ctx *ctx, const tufrg_c64 *P, const tufrg_c64 *C, tufrg_c64 *VP,
                                  tufrg_c64 *VC);

/* Right-hand side dP/dLambda, dC/dLambda [Nq][B][B] at scale lambda.
 * P, C and dP, dC must not overlap. */
tufrg_status tufrg_rhs(tufrg_ctx *ctx, double lambda, const tufrg_c64 *P, const tufrg_c64 *C, tufrg_c64 *dP,
                       tufrg_c64 *dC);

typedef struct {
  double lambda0, lambda_end; /* flow from lambda0 down to lambda_end > 0 */
  int32_t n_steps;            /* > 0: explicit Euler in Lambda on the log grid
                                 Lambda_i = lambda0 (lambda_end/lambda0)^(i/n); 0: Dormand-Prince 5(4)
                                 in ln Lambda with the error norm
                                 max |err| / (atol + rtol max(|X|, |X_new|)) over real and imaginary
                                 parts, step factor clip(0.9 err^-1/5, 0.2, 5), first |h| = h0 */
  double rtol, atol, h0;
  double v_max;               /* stop when max(|P|, |C|) > v_max */
  uint32_t channel_mask;      /* bit 0: flow P, bit 1: flow C (a masked channel keeps its value) */
  int32_t max_steps;          /* 0: no limit */
  /* optional per-step callback (accepted steps); a nonzero return stops the
   * flow cleanly with the state of that step */
  int32_t (*on_step)(void *user, int32_t step, double lambda, double max_coupling);
  void *user;
  /* Loop surrogate (see tufrg_sur_attach).  surrogate = 1: each right-hand
   * side takes its loops from the attached network, recomputes the plain loops
   * on sample_frac of the coarse q_x rows (at least one row; rows chosen by a
   * counter-based hash of sample_seed and the evaluation index) and replaces
   * the network's values there; if the sampled relative error
   * max|L_net - L| / max|L| (maxima over the sampled blocks) exceeds sur_tol,
   * any network output is not finite, or the current max coupling exceeds
   * plain_above, the plain loops are used everywhere for that evaluation.
   * surrogate = 0: plain loops only. */
  int32_t surrogate;
  double sample_frac, sur_tol, plain_above;
  uint64_t sample_seed;
  /* Euler without surrogate and callback, both channels: graph_steps > 1
   * captures up to that many steps (at most 64) at a time in one HIP graph,
   * launched with one host synchronisation per graph instead of one per
   * step; each step's max coupling goes to its own device slot.  The state
   * at the start of a graph is kept: if a step inside it diverges (or reaches
   * max_steps) the graph's steps are undone and replayed one by one, so the
   * result equals that of direct launches bit for bit.  Needs one more copy
   * of P and C on the device (allocated on first use).  0 or 1: direct
   * launches. */
  int32_t graph_steps;
  /* Batched flows (tufrg_batch_flow) of two-orbital instances without
   * graphs: nonzero runs the loop kernels of all active instances in one
   * fused launch per kernel shape and regulator, between a join and a fork of
   * the batch's streams (each instance with the work items and partial sums
   * of its own launch, so the results are bit-identical); 0 launches each
   * instance's loop kernel on its own stream, where it overlaps the other
   * instances' projections and products (faster on the 32-instance Rashba
   * batch: 37.7 against 44.0 ms per step).  Ignored by the single-context
   * flows. */
  int32_t fused_loops;
} tufrg_flow_opts;

typedef struct {
  double lambda_stop;   /* scale of the returned state */
  double lambda_c;      /* where max(|P|,|C|) crossed v_max, linear in ln Lambda between the
                           bracketing accepted steps; 0 if the flow did not diverge */
  double max_coupling;  /* max(|P|, |C|) of the returned state */
  int32_t diverged, n_steps, n_rhs, n_reject, stopped_by_callback;
  int32_t n_plain;        /* right-hand sides with plain loops everywhere */
  int32_t n_surrogate;    /* right-hand sides with network loops (sampled rows plain) */
  int32_t n_fallback;     /* of n_plain: evaluations where the sampled error exceeded sur_tol */
  double max_sample_err;  /* largest sampled relative error seen */
} tufrg_flow_result;

/* Integrates P, C [Nq][B][B] (device, in place) from opts->lambda0. */
tufrg_status tufrg_flow(tufrg_ctx *ctx, const tufrg_flow_opts *opts, tufrg_c64 *P, tufrg_c64 *C,
                        tufrg_flow_result *result);

/* SU(2)-reduced flow of one orbital per site (Sec. 1 and Sec. 6: the
 * spin-rotation-invariant TU-fRG that the method generalises; Sec. 2 channel
 * definitions, Sec. 3.1 matrix RGE, Sec. 3.3 projections).  With spin
 * indices s the spinful propagators are P = p d13 d24 - p^x d14 d23,
 * p^x^{RR'}(s) = e^{is.R'} p^{R,-R'}(s), and C = c d13 d24 - d d14 d23, so the
 * state is three complex arrays p, c, d [Nq][n_ff][n_ff] (B = n_ff, the
 * spinful B / 4), element [q][R][R'].  The reduced equations (cited, not
 * printed, in the paper; re-derived and pinned against the spinful ones):
 *   dp = -(a~ Lpp a~x + a~x Lpp a~),
 *   dc = 2 (2 c~ Lph c~ - c~ Lph d~ - d~ Lph c~),   dd = -2 d~ Lph d~,
 * a~ = p + v + PC(c) + PD(d), c~ = c + v + CP(p) + CD(d), d~ = d + v + CP(p^x)
 * + CD(c) with the cross projections (i)-(iv) of one orbital and v the onsite
 * coefficient (V0[0] of the model), Lpp, Lph the one-band loops.
 * The context must have n_orb = 1, precision TUFRG_FP64, the temperature or
 * Omega cutoff and the orbital basis (else tufrg_create returns
 * E_UNSUPPORTED); such a context serves tufrg_bubble, tufrg_loops_compact,
 * tufrg_band_data and these calls, and returns E_UNSUPPORTED from the spinful
 * state calls.  All arrays are device memory owned by the caller; the calls
 * run on the context's stream.  Errors: E_INVAL (host pointer, lambda <= 0),
 * E_UNSUPPORTED (a spinful context), E_NOMEM, E_HIP. */
tufrg_status tufrg_su2_rhs(tufrg_ctx *ctx, double lambda, const tufrg_c64 *p, const tufrg_c64 *c, const tufrg_c64 *d,
                           tufrg_c64 *dp, tufrg_c64 *dc, tufrg_c64 *dd);

/* Euler flow of the reduced state p, c, d (device, in place) on the grid of
 * tufrg_flow (opts->n_steps >= 1; lambda0, lambda_end, v_max, max_steps,
 * on_step as there; surrogate, graph_steps > 1 and channel masks other than 3
 * return E_UNSUPPORTED).  The stop test and max_coupling use
 * max(|p|, |c|, |d|), which is max(|P|, |C|) of the spinful state.
 * Synchronises once per step; E_NONFINITE on NaN/Inf. */
tufrg_status tufrg_su2_flow(tufrg_ctx *ctx, const tufrg_flow_opts *opts, tufrg_c64 *p, tufrg_c64 *c, tufrg_c64 *d,
                            tufrg_flow_result *res);

/* Optional per-kernel timing with HIP events recorded on the context stream
 * around the launches of one part of the right-hand side:
 *   TUFRG_TIMER_LOOP     the loop kernel launch (both channels in one launch; with
 *                        TUFRG_BF16X3 one interval per matrix-core launch, one per
 *                        channel and chunk of coarse q)
 *   TUFRG_TIMER_PROJECT  real-space transform, gathers and assembly
 *   TUFRG_TIMER_BUNDLE   the two bundle products
 * tufrg_timing(ctx, 1) synchronises, clears and enables; tufrg_timing_read
 * synchronises and returns the accumulated milliseconds and interval count. */
enum {
  TUFRG_TIMER_LOOP = 0,
  TUFRG_TIMER_PROJECT = 1,
  TUFRG_TIMER_BUNDLE = 2,
  TUFRG_TIMER_SURROGATE = 3,
  TUFRG_TIMER_COUNT = 4
};
tufrg_status tufrg_timing(tufrg_ctx *ctx, int32_t enable);
tufrg_status tufrg_timing_read(tufrg_ctx *ctx, int32_t timer, double *total_ms, int32_t *count);

/* ---------------------------------------------------------------------------
 * Compact loops and the learned loop surrogate.
 *
 * The loops depend on R1 - R2 only: the compact form holds, per channel and
 * coarse q, one block of n_o^4 complex entries for each difference vector dR
 * of the list returned by tufrg_dR (n_dR of them, sorted):
 *     Lc[ch][q][iD][(a*n_o + b)*n_o^2 + c*n_o + d] = L(q)[(R1,a,b),(R2,c,d)]
 * for any R1, R2 with R1 - R2 = dR[iD] (channel 0 = pp, 1 = ph).
 *
 * The surrogate is a multilayer perceptron (tufrg_mlp) with GELU activations
 * after every layer but the last, GELU(x) = x Phi(x).  It maps the features
 *   [sin qx, cos qx, sin qy, cos qy, sin 2qx, cos 2qx, sin 2qy, cos 2qy,
 *    ln(Lambda)/5, ch == 0, ch == 1, one-hot(iD)]   (11 + n_dR values)
 * of a block to Lc / s(Lambda), real and imaginary parts interleaved
 * (2 n_o^4 values), where s(Lambda) is a positive scale given as a table
 * (typically the largest |Lc| at that scale) and interpolated linearly in
 * (ln Lambda, ln s).  The paper has no learned component; this
 * accelerates the loops of Sec. 3.1 / Sec. 4.2 and is always checked against
 * them during a flow (tufrg_flow_opts.surrogate). */

/* Compact loops of both channels at lambda (deriv as in tufrg_bubble):
 * device [2][Nq][n_dR][n_o^4] tufrg_c64. */
tufrg_status tufrg_loops_compact(tufrg_ctx *ctx, double lambda, int32_t deriv, tufrg_c64 *Lc);
/* The difference vectors of the compact blocks: host [n_dR][2]. */
tufrg_status tufrg_dR(const tufrg_ctx *ctx, int32_t *dR);

/* Surrogate network.  sizes[0..n_sizes): input, hidden..., output widths.
 * params: host array of the initial parameters (per layer W[out][in]
 * row-major, then b[out]), or NULL for zeros; float32. */
typedef struct tufrg_mlp tufrg_mlp;
tufrg_status tufrg_mlp_create(int32_t n_sizes, const int32_t *sizes, const float *params, void *stream,
                              tufrg_mlp **out);
tufrg_status tufrg_mlp_destroy(tufrg_mlp *net);
const char *tufrg_mlp_last_error(const tufrg_mlp *net);
tufrg_status tufrg_mlp_n_params(const tufrg_mlp *net, int64_t *n);
/* copy parameters out to / in from device memory (set also resets Adam) */
tufrg_status tufrg_mlp_params(tufrg_mlp *net, float *params);
tufrg_status tufrg_mlp_set_params(tufrg_mlp *net, const float *params);
/* Y[n][n_out] = net(X[n][n_in]); device arrays */
tufrg_status tufrg_mlp_forward(tufrg_mlp *net, int64_t n, const float *X, float *Y);
/* mean squared error over the batch and outputs and its gradient with respect
 * to the parameters (device, n_params floats; NULL: internal buffer used by
 * tufrg_mlp_adam_step with grad = NULL); loss: host, may be NULL.  n <= 65536. */
tufrg_status tufrg_mlp_loss_grad(tufrg_mlp *net, int32_t n, const float *X, const float *T, float *grad,
                                 double *loss);
/* Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) with learning rate lr */
tufrg_status tufrg_mlp_adam_step(tufrg_mlp *net, const float *grad, float lr);
/* epochs of shuffled minibatch Adam over rows X[n], T[n] (device); the mean
 * batch loss of the last epoch is returned in last_epoch_loss (host, may be NULL) */
tufrg_status tufrg_mlp_train(tufrg_mlp *net, int64_t n, const float *X, const float *T, int32_t batch,
                             int32_t epochs, float lr, uint64_t seed, double *last_epoch_loss);

/* Features and targets of n blocks (q, ch, iD device int32 lists); with all
 * three lists NULL the blocks are all 2 Nq n_dR in compact order.
 * X: device [n][11 + n_dR] at lambda; T: device [n][2 n_o^4] = Lc / scale
 * from Lc (device [2][Nq][n_dR][n_o^4]); max_abs (host, may be NULL) returns
 * the largest |Lc| over the listed blocks.  Invalid block indices give NaN
 * targets. */
tufrg_status tufrg_sur_features(tufrg_ctx *ctx, int64_t n, const int32_t *q, const int32_t *ch, const int32_t *iD,
                                double lambda, float *X);
tufrg_status tufrg_sur_targets(tufrg_ctx *ctx, int64_t n, const int32_t *q, const int32_t *ch, const int32_t *iD,
                               double scale, const tufrg_c64 *Lc, float *T, double *max_abs);
/* Attach a network (NULL detaches; the context does not own it) with its
 * target scale table (host arrays of n_scale positive lambda and s values).
 * Input width must be 11 + n_dR, output 2 n_o^4, and the network must have
 * been created on the context's stream. */
tufrg_status tufrg_sur_attach(tufrg_ctx *ctx, tufrg_mlp *net, int32_t n_scale, const double *lambda,
                              const double *scale);
/* Compact loops of both channels from the attached network (as tufrg_loops_compact). */
tufrg_status tufrg_sur_loops(tufrg_ctx *ctx, double lambda, tufrg_c64 *Lc);

/* ---------------------------------------------------------------------------
 * Batches of independent instances (several models, form-factor sets and
 * meshes at once).  Each instance is a context as above; the batch runs them
 * on n_streams concurrent streams (default priority) and steps all of them in
 * lockstep on one Euler grid, with one host synchronisation per step for all
 * stop tests.  An instance that diverges stops; the others continue. */
typedef struct tufrg_batch tufrg_batch;
tufrg_status tufrg_batch_create(int32_t n_inst, const tufrg_model *models, const tufrg_setup *setups,
                                int32_t n_streams, tufrg_batch **out);
tufrg_status tufrg_batch_destroy(tufrg_batch *batch);
const char *tufrg_batch_last_error(const tufrg_batch *batch);
tufrg_status tufrg_batch_dims(const tufrg_batch *batch, int32_t inst, int32_t *B, int32_t *Nq, int32_t *Nf,
                              int32_t *n_dR);
/* P[i], C[i]: device [Nq_i][B_i][B_i] of instance i, integrated in place;
 * results[i] per instance.  opts->n_steps must be > 0 (Euler) and
 * opts->surrogate 0; the callback is not used.  The call synchronises the
 * device before it starts and all its streams when it returns. */
tufrg_status tufrg_batch_flow(tufrg_batch *batch, const tufrg_flow_opts *opts, tufrg_c64 *const *P,
                              tufrg_c64 *const *C, tufrg_flow_result *results);

#ifdef __cplusplus
}
#endif

#endif /* TUFRG_H */

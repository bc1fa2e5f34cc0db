// Host-side launchers of the TU-fRG kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>

namespace tufrg {

// a0: band data on the fine mesh (eigenvalues minus mu, packed projectors)
// unit_pi: band basis, Pi_m(k) = e_m e_m^T (eigenvalues as always)
hipError_t launch_band(int n_o, int Lf, int n_hop, const int *hop_R, const double *hop_t, double mu, int unit_pi,
                       double *e, double *pi, float *e32, float *pi32, hipStream_t st);
hipError_t launch_kval(int n, int Nf, int aos_no, const double *e, double lam, int scheme, int deriv, double *kv,
                       float *kv32, hipStream_t st);
// two orbitals: ekv[k] = (e_0, e_1, K(e_0), K(e_1)) and the static pi4[k], k-major 4-vectors
hipError_t launch_ekv4(int Nf, const double *band, double lam, int scheme, int deriv, double *ekv, float *ekv32,
                       hipStream_t st);
hipError_t launch_pi4(int Nf, const double *band, double *pi4, float *pi4_32, hipStream_t st);
// shell scheme: factors (a, b) of every band value e[m][k] (component-major);
// two orbitals [Nf][4] = (a_0, a_1, b_0, b_1), more orbitals [Nf][n_o][2]
hipError_t launch_shell_ab(int n_o, int Nf, const double *e, double lam, int deriv, double *cv, float *cv32,
                           hipStream_t st);
// component-major [nc][Nf] -> k-major [Nf][nc] (FP64 and FP32)
hipError_t launch_to_kmajor(int nc, int Nf, const double *src, double *dst, float *dst32, hipStream_t st);

// a1-a3: form-factor projected orbital loops
struct LoopArgs {
  int n_o, Lq, n_ref, Lf, Nq;
  int ndx, ndy;        // computed box: dx in [0, ndx), dy in [-ndy, ndy]
  int nkyb, nkxc;      // ky blocks of 64 lanes, kx chunks
  int kxr = 2;         // six spin-orbitals on the matrix cores: kx rows per work item (1..8)
  int ch_first, n_ch;  // channels 0 (pp) and/or 1 (ph)
  int q_first, n_q;    // coarse q range
  const int *rows = nullptr;  // if set: q = whole q_x rows rows[0 .. n_q / Lq) (q_first unused)
  int scheme, deriv, prec;
  double lam;
  const void *band;    // band data (FP64 or FP32 by prec): two orbitals component-major
                       // [n_o + n_o^3][Nf], more orbitals k-major [Nf][n_o + n_o^3]
  const void *kv;      // regulator values, [n_o][Nf] or [Nf][n_o] like the band data
  const double *tw;    // exp(-2 pi i j / Lf), [Lf][2]
  const float *tw32 = nullptr;  // the same in FP32
  void *partial;       // [n_ch][n_q][nkyb * nkxc][ndx][2 ndy + 1][n_o^4][2] in the arithmetic type
                       // (FP64 for TUFRG_FP64, else FP32: the partials carry no more)
  const int *pairs = nullptr;  // more than two orbitals: [n_pairs][2] entry and its conjugate partner
  int n_pairs = 0;
  const void *phy = nullptr;   // more than two orbitals: exp(-2 pi i ky dy / Lf), [Lf][ndy][2], like band
  const void *ekv = nullptr;   // two orbitals: [Nf][4] = (e_0, e_1, K(e_0), K(e_1)), like band
  const void *pi4 = nullptr;   // two orbitals: [Nf][4] = (Pi_0[00], Pi_0[11], Re Pi_0[01], Im Pi_0[01])
  const void *cv = nullptr;    // shell scheme: shell factors, two orbitals [Nf][4] = (a_0, a_1, b_0, b_1),
                               // more orbitals [Nf][n_o][2] = (a_m, b_m); like band
  int pair = 0;                // six spin-orbitals on the matrix cores: bands (0,1), (2,3), (4,5)
                               // degenerate at every k, summed by pairs
  const float *pir = nullptr;     // with pair: [Nf][3][36] pair sums of the packed projectors (FP32)
  const double *pir64 = nullptr;  // the same in FP64 (six spin-orbitals on the vector units, FP64)
};
hipError_t launch_loop(const LoopArgs &a, hipStream_t st);
// several two-orbital instances of one precision in fused launches (one per
// kernel shape and regulator): instance i sums both channels over all its
// coarse q into a[i].partial, with the work items of its own launch_loop.
// desc_h (pinned host) and desc_d (device) hold n descriptors; desc_h is
// rewritten, so the previous call's copies must be complete.
struct No2Inst {
  const void *ekv, *pi4, *cvp, *twk;
  const double *tw;
  void *partial;
  double lam;
  int Lq, n_ref, Lf, nkyb, nkxc, kxper, n_q, deriv, item0, pad;
};
hipError_t launch_loop_batch(const LoopArgs *a, int n, No2Inst *desc_h, No2Inst *desc_d, hipStream_t st);
// more than two spin-orbitals (six: t2g with spin-orbit coupling)
hipError_t launch_loop_gen(const LoopArgs &a, hipStream_t st);
// six spin-orbitals on the matrix cores in the real basis of Hermitian
// matrices (one channel): row buffers Y of loop_rb_rowbuf_floats(ndy, Lf)
// floats per group of four coarse q, then (sums) the compact loops; the
// half-plane points of the computed shape from loop_rb_half_points.  The A
// operand (phases times projectors, split; independent of q, Lambda and the
// channel) is computed once into loop_rb_apre_bytes(ndy, Lf) bytes.
size_t loop_rb_apre_bytes(int ndy, int Lf, int pair);
hipError_t launch_loop_rb_apre(int ndy, int pair, const float *band, const float *pir, const float *phy, int Lf,
                               void *apre, hipStream_t st);
// pair sums of the packed projectors into pir (FP32) and/or pir64 (FP64; either may be null)
hipError_t launch_pair_pi(int Nf, const double *band, float *pir, double *pir64, hipStream_t st);
hipError_t launch_loop_rb(const LoopArgs &a, int ch, const void *apre, float *Y, hipStream_t st);
hipError_t launch_loop_rb_sums(const LoopArgs &a, const float *Y, double *lamb, const int *hmap, int nD,
                               double *dst, hipStream_t st);
size_t loop_rb_rowbuf_floats(int ndy, int Lf);
int loop_rb_half_points(int ndy, int *dx, int *dy);
// sums partials, applies 1/Nf, fills dx < 0 by hermiticity
hipError_t launch_loop_finalize(const LoopArgs &a, int nD, const int *dlist, double *compact, hipStream_t st);
// compact [n_ch][n_q][nD][n_o^4] -> full [n_q][B][B] for one channel
hipError_t launch_loop_expand(int n_o, int n_ff, int nD, int n_q, const int *didx, const double *compact,
                              double *out, hipStream_t st);

// a4-a5: real-space transform, gathers, assembly of projected vertices
struct ProjArgs {
  int n_o, n_ff, B, Lq, Nq, nD;
  const int *dlist;    // [nD][2]
  const int *ffgrid;   // [17][17] form-factor index of (x, y) in [-8, 8]^2, -1 outside S
  const int *dgrid;    // [17][17] index into dlist, -1 outside D
  const int *ff;       // [n_ff][2]
  const double *twq;   // exp(+2 pi i j / Lq), [Lq][2]
  int ny;              // distinct rho_y over dlist (at most 9)
  const double *phy;   // exp(+2 pi i qy y_s / Lq) of those values y_s, [Lq][ny][2]
  const int *dtab;     // per rho of dlist: (rho_x mod Lq) | (slot s of rho_y) << 16
  const int *dslot;    // [9][9] per slot s the rho of D with rho_y = y_s: iD | (rho_x mod Lq) << 16, else -1
};
// ws: workspace of ws_doubles >= proj_ws_row_doubles (one qx row of the
// two-stage transforms; more rows per pass with more)
size_t proj_ws_row_doubles(const ProjArgs &a);
hipError_t launch_ft(const ProjArgs &a, const double *P, const double *C, double *ws, size_t ws_doubles,
                     double *real, hipStream_t st);
hipError_t launch_gather(const ProjArgs &a, const double *real, double *G, hipStream_t st);
// D [Nq][B][B] (layout of C) from C: D_{n1n2n3n4} = -C_{n1n2n4n3}
hipError_t launch_channel_d(int n_o, int B, int Nq, const double *C, double *D, hipStream_t st);
// nw = 1: only VP from P and G[0]
hipError_t launch_assemble(const ProjArgs &a, const double *P, const double *C, const double *G,
                           const double *v0p, const double *v0c, double *VP, double *VC, double *ws,
                           size_t ws_doubles, hipStream_t st, int nw = 2);

// a6: bundle products  out = f * V L V  per q, L expanded from compact form;
// bundles larger than 64 need a workspace tmp of n_q * B * B complex
hipError_t launch_bundle(int prec, int n_o, int n_ff, int B, int nD, int n_q, const int *didx, const double *V,
                         const double *Lc, double factor, double *out, double *tmp, hipStream_t st);
// the same on the matrix cores with BF16 split operands (k_bundle_mfma.hip), in
// chunks of q that fit the workspace ws (at least bundle_split_bytes_per_q(B))
size_t bundle_split_pad(int B);
size_t bundle_split_bytes_per_q(int B);
hipError_t launch_bundle_bf16x3(int n_o, int n_ff, int B, int nD, int n_q, const int *didx, const double *V,
                                const double *Lc, double factor, double *out, void *ws, size_t ws_bytes,
                                hipStream_t st);

// SU(2)-reduced flow of one orbital (k_su2.hip): one-band loops into compact
// [n_ch][n_q][nD] complex; X -> X^x; the gathers G[3][nD][B][B] of a~, c~, d~
// from rA = (p, c)(rho), rB = (p^x, d)(rho); the reduced products per q (B <= 25)
// (the kx range in nkxc chunks, partial sums in part of loop1_partial_doubles)
size_t loop1_partial_doubles(int n_q, int nD, int nkxc);
hipError_t launch_loop1(int Lq, int n_ref, int nD, const int *dlist, const double *e, const double *kv,
                        const double *tw, double lam, int scheme, int deriv, int ch_first, int n_ch, int q_first,
                        int n_q, int nkxc, double *part, double *out, hipStream_t st);
hipError_t launch_su2_exch(int n_ff, int Nq, int Lq, const int *ff, const int *fneg, const double *twq,
                           const double *X, double *Xx, hipStream_t st);
hipError_t launch_su2_gather(int B, int nD, const int *ff, const int *dlist, const int *ffgrid, const int *dgrid,
                             const double *rA, const double *rB, double *G, hipStream_t st);
hipError_t launch_su2_bundle(int B, int Nq, int nD, const int *didx, const double *Lc, const double *Va,
                             const double *Vax, const double *Vc, const double *Vd, double f, double *dp, double *dc,
                             double *dd, hipStream_t st);

// orbital <-> band basis (k_basis.hip): compact basis matrix [Nq][nD][n_o^4] of one
// channel (0: pp, U matrix; 1: ph, X matrix) from U[Nf][n_o][n_o] (orbital rows, band
// columns); box: D inside [-box, box]^2 (2 or 4); dlist [nD][2]; tw = exp(-2 pi i j /
// Lf), [Lf][2]; rows: workspace of basis_rows_doubles(n_o, Lf, box, q_chunk) doubles
// (the coarse q are processed q_chunk at a time)
size_t basis_rows_doubles(int n_o, int Lf, int box, int nq);
hipError_t launch_basis_compact(int channel, int n_o, int Lq, int n_ref, int nD, int box, const int *dlist,
                                const double *U, const double *tw, double *rows, int q_chunk, double *out,
                                hipStream_t st);
// Y[q] = (A (x) 1) X[q] (A (x) 1)^H in the form-factor index, A [n_ff][n_ff] complex on the device
hipError_t launch_ff_apply(int n_ff, int no2, int n_q, const double *A, const double *X, double *Y, hipStream_t st);
// C[q] = opA(A[q]) opB(B[q]), n x n complex, op 1 = conjugate transpose (not both)
hipError_t launch_zgemm_batched(int n, int n_q, int opA, int opB, const double *A, const double *Bm, double *C,
                                hipStream_t st);

// a7: ODE updates and reductions
hipError_t launch_axpy_max(long long n, const double *x, double h, const double *dx, double *y,
                           unsigned long long *maxbits, unsigned int *flag, hipStream_t st);
hipError_t launch_lincomb(long long n, const double *x, int nk, const double *const *k, const double *coef,
                          double h, double *y, hipStream_t st);
hipError_t launch_dp_error(long long n, const double *x0, const double *x1, int nk, const double *const *k,
                           const double *ecoef, double h, double rtol, double atol, unsigned long long *errbits,
                           unsigned int *flag, hipStream_t st);
hipError_t launch_clear_reduce(unsigned long long *bits, unsigned int *flag, hipStream_t st);
hipError_t launch_scale(long long n, const double *x, double s, double *y, hipStream_t st);
// y = a + b over n doubles (n even: complex arrays)
hipError_t launch_add(long long n, const double *a, const double *b, double *y, hipStream_t st);

// loop surrogate network (k_mlp.hip)
hipError_t launch_gemm_f32(int M, int N, int K, const float *A, int lda, int tA, const float *B, int ldb, int tB,
                           const float *bias, int epi, float *C, int ldc, float *Z, hipStream_t st);
hipError_t launch_gelu_bwd(long long n, const float *Z, float *dA, hipStream_t st);
// part: workspace of ceil(rows / 64) * cols floats
hipError_t launch_colsum(int rows, int cols, const float *dZ, float *part, float *db, hipStream_t st);
hipError_t launch_mse_grad(long long n, const float *Y, const float *T, float *dY, double *loss, hipStream_t st);
hipError_t launch_adam(long long n, float *p, const float *g, float *m, float *v, float lr, float b1, float b2,
                       float eps, int t, hipStream_t st);
hipError_t launch_gather_rows(int rows, int len, const int *idx, const float *src, float *dst, hipStream_t st);
hipError_t launch_sur_features(long long n, const int *ql, const int *cl, const int *dl, int Lq, int nD, double lam,
                               float *X, hipStream_t st);
hipError_t launch_sur_targets(long long n, const int *ql, const int *cl, const int *dl, int Nq, int nD, int no4,
                              double s, const double *Lc, float *T, hipStream_t st);
hipError_t launch_sur_scatter(long long n, int no4, double s, const float *Y, double *Lc, unsigned int *bad,
                              hipStream_t st);
hipError_t launch_sur_compare(long long n, const double *a, const double *b, unsigned long long *bits,
                              hipStream_t st);
hipError_t launch_absmax_f32(long long n, const float *x, unsigned int *bits, hipStream_t st);

}  // namespace tufrg

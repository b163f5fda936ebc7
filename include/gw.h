/*
 * gw.h -- C ABI of libgwspinor: the Epsilon-stage hot path of fully
 * relativistic (two-component spinor) GW on one AMD Instinct MI355X (gfx950).
 *
 * The operations follow Sec. II of arXiv:2206.00808 ("Spinor Wavefunctions in
 * Many-Body Perturbation Theory"):
 *   M_vc(q+G)   = sum_alpha <v,k+q,alpha| e^{i(q+G).r} |c,k,alpha>
 *                 computed by transforming the spin-summed real-space product
 *                 (the matrix-element definition and Eq. (matrix_el));
 *   chi0_GG'    = (1/N_k) sum_{v,c} M*_vc(G) M_vc(G') [Adler-Wiser bracket]
 *                 on the imaginary axis w = i*omega, eta = 0
 *                 (the polarizability P_GG'(q,w));
 *   eps_GG'     = delta_GG' - v(q+G) chi0_GG'  and its inverse
 *                 (the dielectric-matrix definition; the Performance section
 *                 names the inversion as a large share of Epsilon's time).
 *
 * Conventions shared by every entry point
 *   - Energies in Hartree.  G vectors are integer triples g (the Cartesian
 *     vector is 2*pi*(g + k)/a on an orthorhombic cell; the library never needs a).
 *   - Complex numbers are interleaved (re, im).  GW_C128 = two doubles,
 *     GW_C64 = two floats.  All arrays are row-major, last index fastest.
 *   - "(device)" pointers are HIP device memory owned by the caller; the
 *     library never frees or retains them past the call.  "(host)" pointers are
 *     read during the call only.
 *   - Every call is enqueued on the context's HIP stream and is asynchronous
 *     with respect to the host unless stated otherwise.
 *   - Arguments are validated on the host before anything is enqueued; on an
 *     error status no output has been touched.  gw_last_error() returns a
 *     per-context message describing the last non-OK status.
 *   - A context is not thread-safe; use one context per host thread.
 *   - Contexts allocate their own device workspace (grown on demand, freed by
 *     gw_ctx_destroy).  Calls overlapping on one context race on it.
 */
#ifndef GW_SPINOR_H
#define GW_SPINOR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GW_OK = 0,
  GW_EINVAL = -1,        /* bad argument (size, null pointer, enum value) */
  GW_ENOMEM = -2,        /* device workspace allocation failed */
  GW_EDEVICE = -3,       /* no usable HIP device, or a HIP runtime error */
  GW_EALIAS = -4,        /* FFT box too small: the pair product aliases onto an eps G */
  GW_ESINGULAR = -5,     /* a zero pivot in the LU factorisation of eps */
  GW_ENOTTRAINED = -6,   /* closure inference requested from an untrained network */
  GW_EUNSUPPORTED = -7,  /* valid request this build does not implement */
  GW_EFALLBACK = 1       /* not an error: the closure fell back to the full band sum */
} gw_status;

typedef enum { GW_C128 = 0, GW_C64 = 1 } gw_dtype;

/* Contraction precision for chi0 (gw_chi0_accumulate):
 *   GW_PREC_FP64      complex double products, double accumulation;
 *   GW_PREC_SPLITBF16 each float component x is split into hi = bf16(x) and
 *                     lo = bf16(x - hi) (round to nearest even); every real
 *                     product is hi*hi + hi*lo + lo*hi on BF16 matrix cores with
 *                     float accumulation inside a K-chunk, chunks summed in double.
 *                     Requires GW_C64 matrix elements.                            */
typedef enum { GW_PREC_FP64 = 0, GW_PREC_SPLITBF16 = 1 } gw_prec;

typedef struct gw_ctx gw_ctx;

/* Create a context on HIP device `device`; `hip_stream` is a hipStream_t (may be
 * NULL = the null stream).  Returns GW_EDEVICE when no device is usable. */
gw_status gw_ctx_create(gw_ctx** ctx, int device, void* hip_stream);
gw_status gw_ctx_destroy(gw_ctx* ctx);
/* Change the stream later calls are enqueued on. */
gw_status gw_ctx_set_stream(gw_ctx* ctx, void* hip_stream);
/* Message for the last non-OK status on this context ("" if none).  The string
 * is owned by the context and valid until its next call. */
const char* gw_last_error(const gw_ctx* ctx);
/* Static name of a status code. */
const char* gw_status_string(gw_status s);

/* Per-kernel timing.  When enabled, every kernel the library launches is
 * bracketed by HIP events on the stream it runs on; gw_ctx_profile_entry
 * synchronises the stream and reports, per kernel name, the launch count and
 * the summed event time in milliseconds.  Disabled by default.
 * gw_ctx_profile_only restricts the events to the kernels of one name (NULL:
 * all), so that a timed run carries events around that kernel only; events
 * between short dependent kernels lengthen the gaps between them. */
gw_status gw_ctx_profile(gw_ctx* ctx, int enable);
gw_status gw_ctx_profile_only(gw_ctx* ctx, const char* name);
gw_status gw_ctx_profile_reset(gw_ctx* ctx);
int gw_ctx_profile_count(gw_ctx* ctx);
gw_status gw_ctx_profile_entry(gw_ctx* ctx, int i, const char** name, int* launches,
                               double* total_ms);

/*
 * gw_mtxel_spinor -- plane-wave matrix elements of a spinor band pair
 * (Sec. II, definition of M_nn'(k,q,G) and Eq. (matrix_el)).
 *
 * For every valence band v at k+q and conduction band c at k:
 *   u_n^s(r_j) = sum_{G in sphere} c_n^s(G) exp(+2 pi i g.j/n)          (band to grid)
 *   rho_vc(r)  = sum_{s=1..nspinor} conj(u_v^s(r)) u_c^s(r)            (spin-summed product)
 *   M_vc(G)    = (1/N) sum_j rho_vc(r_j) exp(+2 pi i g.j/n),  G in geps (pruned transform)
 * The spin sum is taken before the transform; by linearity this equals the
 * paper's per-spin transforms followed by the spin sum.
 *
 *   box        (host) int[3] FFT grid n1 x n2 x n3; each n_i must factor into 2, 3, 5.
 *   nspinor    1 (spinless) or 2 (spinor).
 *   nv, ngv    valence band count and wavefunction-sphere size at k+q.
 *   gv         (host) int32[ngv][3] G vectors of the k+q sphere.
 *   cv         (device) complex[nv][nspinor][ngv] coefficients, dtype `dtype`.
 *   nc, ngc, gc, cc   the same for the conduction bands at k.
 *   neps       size of the dielectric sphere;  geps (host) int32[neps][3].
 *   dtype      GW_C128 (double transforms) or GW_C64 (float transforms).
 *   mtxel      (device) out complex[nv][nc][neps], dtype `dtype`; pair p = v*nc + c.
 *   head_index index of G = 0 in geps for the small-q head, or -1.
 *   mhead      (device) out complex double[nv*nc]: M_vc(G=0) by the direct
 *              double-precision overlap sum_s sum_G conj(c_v^s(G)) c_c^s(G); NULL to skip.
 * Errors: GW_EINVAL (sizes, a G vector outside the box, duplicate G), GW_EALIAS
 * when some n_i <= max|gv_i| + max|gc_i| + max|geps_i|, GW_ENOMEM.
 */
gw_status gw_mtxel_spinor(gw_ctx* ctx, const int box[3], int nspinor,
                          int nv, int ngv, const int32_t* gv, const void* cv,
                          int nc, int ngc, const int32_t* gc, const void* cc,
                          int neps, const int32_t* geps, gw_dtype dtype,
                          void* mtxel, int head_index, double* mhead);

/*
 * gw_chi0_accumulate -- chi0_f[G][G'] += prefactor * sum_p w_p(omega_f) conj(M_p(G)) M_p(G')
 * (Sec. II, the Adler-Wiser polarizability at imaginary frequency, eta = 0):
 *   w_p(omega) = 1/(D_p - i omega) + 1/(D_p + i omega) = 2 D_p / (D_p^2 + omega^2),
 *   D_p = ev[v] - ec[c],  p = v*nc + c.
 *
 *   mtxel      (device) complex[nv*nc][neps] of dtype `dtype` (as written by gw_mtxel_spinor).
 *   ev, ec     (device) double[nv], double[nc].
 *   nfreq      number of frequencies; omega (host) double[nfreq], each >= 0 (0 = static).
 *   prefactor  1/N_k.
 *   prec       GW_PREC_FP64 (any dtype; c64 inputs are widened) or GW_PREC_SPLITBF16 (c64 only).
 *   mhead      (device) complex double[nv*nc] FP64 head elements or NULL; when given
 *              together with head_index >= 0, row and column head_index of chi0
 *              are accumulated in double from mhead (head) and mhead x mtxel (wings).
 *   chi0       (device) in/out complex double[nfreq][neps][neps]; the update is added.
 * chi0's update is Hermitian; only upper tiles are computed and mirrored.
 */
gw_status gw_chi0_accumulate(gw_ctx* ctx, int nv, int nc, int neps,
                             const void* mtxel, gw_dtype dtype,
                             const double* ev, const double* ec,
                             int nfreq, const double* omega, double prefactor,
                             gw_prec prec, const double* mhead, int head_index,
                             double* chi0);

/*
 * gw_chi0_accumulate_noalloc -- gw_chi0_accumulate in FP64 (GW_PREC_FP64)
 * without any allocation, for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid it.
 * Same arguments and result as gw_chi0_accumulate with prec = GW_PREC_FP64;
 * the contraction runs as one pair range (no partial sums), the frequencies
 * travel by value in the kernel arguments, and the pair weights live in a
 * fixed 32 MiB device array of the library (one copy on each device, held until
 * the process ends).  Limits: nfreq <= 64 and nfreq * nv * nc * 8 bytes <= 32
 * MiB, else GW_EINVAL before anything is enqueued.  Calls that overlap on one
 * device share that array and race; calls on one stream are ordered.
 * Asynchronous; calls no allocating routine.
 */
gw_status gw_chi0_accumulate_noalloc(gw_ctx* ctx, int nv, int nc, int neps,
                                     const void* mtxel, gw_dtype dtype, const double* ev,
                                     const double* ec, int nfreq, const double* omega,
                                     double prefactor, const double* mhead, int head_index,
                                     double* chi0);

/*
 * gw_head_dipole -- the q -> 0 head M_vc(q, G=0) from momentum matrix elements at
 * one k-point (Sec. II, optical absorption: the dipole relation with the
 * momentum operator standing in for the velocity), to first order in q:
 *   mhead[v*nc + c] = q.P_vc / (E_v - E_c),
 *   P_vc = sum_s sum_G conj(c_v^s(G)) (k+G) c_c^s(G),  k+G = (g + kpt) 2 pi / cell.
 * No wavefunctions at k+q are needed.  The result is the mhead input of
 * gw_chi0_accumulate (valence and conduction here both at k).
 *   g        (host) int32[ng][3] G-vectors shared by cv and cc.
 *   cv, cc   (device) complex[nv][nspinor][ng], complex[nc][nspinor][ng] of dtype.
 *   cell     (host) double[3] orthorhombic cell edges (bohr); kpt (host) double[3]
 *            reduced k; qcart (host) double[3] the small q in Cartesian bohr^-1.
 *   ev, ec   (device) double[nv], double[nc].
 *   mhead    (device) out complex double[nv*nc]; pairs with ev == ec give
 *            non-finite values.
 * Errors: GW_EINVAL for nspinor not 1 or 2, negative sizes, unknown dtype, NULL
 * arrays, a non-positive cell edge or non-finite k or q.
 */
gw_status gw_head_dipole(gw_ctx* ctx, int nspinor, int nv, int nc, int ng, const int* g,
                         const void* cv, const void* cc, gw_dtype dtype, const double* cell,
                         const double* kpt, const double* qcart, const double* ev,
                         const double* ec, double* mhead);

/*
 * gw_chi0_accumulate_real -- the polarizability on the real frequency axis with
 * broadening (Sec. II, the Adler-Wiser sum as written):
 *   chi0_f[G][G'] += prefactor * sum_p b_p(omega_f) conj(M_p(G)) M_p(G'),
 *   b_p(omega) = 1/(D_p - omega + i eta) + 1/(D_p + omega + i eta),  D_p = ev[v] - ec[c].
 * The update is not Hermitian. It is formed as A + iB from two Hermitian
 * contractions with the real weights Re b and Im b, each computed like
 * gw_chi0_accumulate's.
 *   omega (host) double[nfreq], any finite real frequencies; eta > 0.
 *   chi0  (device) in/out complex double[nfreq][neps][neps]; the update is added.
 *   The other arguments are as for gw_chi0_accumulate; there is no head/wings
 *   split (the q -> 0 head is an imaginary-axis quantity here).
 * Uses 2*nfreq*neps^2*16 bytes of context workspace for A and B.
 * Errors: GW_EINVAL for eta <= 0, non-finite omega or prefactor, NULL arrays,
 * unknown dtype/precision, split-BF16 with GW_C128, nfreq > 32767.
 */
gw_status gw_chi0_accumulate_real(gw_ctx* ctx, int nv, int nc, int neps,
                                  const void* mtxel, gw_dtype dtype,
                                  const double* ev, const double* ec,
                                  int nfreq, const double* omega, double eta,
                                  double prefactor, gw_prec prec, double* chi0);

/*
 * gw_epsinv -- eps_f = I - diag(vcoul) chi0_f and eps_f^-1, all in double
 * (Sec. II, dielectric matrix and W = eps^-1 v).  When v > 0 and chi0 is
 * Hermitian negative semidefinite (the imaginary axis), eps~ = I - V^1/2 chi0
 * V^1/2 is Hermitian positive definite and is inverted by blocked Gauss-Jordan
 * without pivoting, every pivot checked (real part >= 1/2, |imaginary part| <=
 * 1/4 of it), and chi0 checked for Hermiticity as eps~ is formed
 * (|chi_ij - conj(chi_ji)| <= 1e-12 (|chi_ij| + |chi_ji|)).  If a check fails
 * (for example eps from the real axis), the
 * Gauss-Jordan result is kept only if max_ij |(eps X - I)_ij| <= 1e-10 / neps
 * (|re| + |im|, every frequency, eps formed again and multiplied on the matrix
 * cores), which bounds the relative error of X in the infinity norm by 1e-10;
 * otherwise, and whenever some v <= 0, the whole call is redone by
 * gw_epsinv_lu's LU path.
 *
 *   chi0    (device) complex double[nfreq][neps][neps].
 *   vcoul   (device) double[neps], v(q+G) = 4 pi / (Omega |q+G|^2).
 *   epsinv  (device) out complex double[nfreq][neps][neps]; may not alias chi0.
 * Synchronises the context stream to read the flags: GW_EINVAL if chi0 holds
 * a non-finite entry, GW_ESINGULAR if any pivot of the LU path was exactly zero
 * (epsinv then holds non-finite values).
 */
gw_status gw_epsinv(gw_ctx* ctx, int neps, int nfreq, const double* chi0,
                    const double* vcoul, double* epsinv);

/*
 * gw_epsinv_lu -- eps_f^-1 for any nonsingular eps_f (for example from
 * gw_chi0_accumulate_real), by LU factorisation with partial pivoting (row
 * interchanges, largest |re|+|im| in the column, lowest index on ties) and
 * forward and back substitution on the permuted identity, in double.
 * Arguments, ownership and errors as for gw_epsinv.
 */
gw_status gw_epsinv_lu(gw_ctx* ctx, int neps, int nfreq, const double* chi0,
                       const double* vcoul, double* epsinv);

/*
 * gw_epsinv_lowrank -- eps^-1 in a reduced basis of nb static eigenvectors
 * (Sec. IV, Bi2Se3: the full-frequency calculation keeps 200 eigenvectors,
 * about a tenth of the spectrum).  With epst(w) = I - V^1/2 chi0(w) V^1/2 and U the
 * eigenvectors of epst(0) with the nb largest eigenvalues:
 *   epst^-1(w) ~= I + U ((U^H epst(w) U)^-1 - I) U^H,  eps^-1 = V^1/2 epst^-1 V^-1/2.
 * The eigenvectors come from a cyclic Jacobi method on the GPU (converged to an
 * off-diagonal norm of 1e-14 of the matrix's); nb = neps gives the exact inverse.
 *   chi0  (device) complex double[nfreq][neps][neps], Hermitian, frequency 0 first.
 *   vcoul (device) double[neps], every entry > 0.
 *   epsinv (device) out complex double[nfreq][neps][neps], not chi0.
 *   eigenvalues (device) out double[neps] of epst(0) in ascending order, or NULL.
 * Allocates its own buffers (about 16 (nfreq + 2) neps^2 bytes) and synchronises
 * the context stream.
 * Errors: GW_EINVAL for negative sizes, nb outside 1..neps, neps > 8192, NULL
 * arrays, aliasing, vcoul <= 0, non-finite input; GW_ENOMEM; GW_ESINGULAR from
 * the small inverses.
 */
gw_status gw_epsinv_lowrank(gw_ctx* ctx, int neps, int nfreq, const double* chi0,
                            const double* vcoul, int nb, double* epsinv, double* eigenvalues);

/*
 * The reduced basis in three steps, for chi0 built directly in it (the use the
 * scheme is for: P nb^2 instead of P N^2 work and nb^2 memory per frequency):
 *
 * gw_lowrank_basis -- U (device out complex double[neps][nb], columns the
 *   eigenvectors of epst(0) = I - V^1/2 chi0(0) V^1/2 with the nb largest
 *   eigenvalues, descending) from the static chi0 (device complex double
 *   [neps][neps], Hermitian) by the Jacobi method of gw_epsinv_lowrank;
 *   eigenvalues (device out double[neps], ascending) or NULL.  Allocates its own
 *   buffers and synchronises the context stream.  GW_EINVAL for nb outside
 *   1..neps, neps > 8192, NULL arrays, vcoul <= 0, non-finite input.
 * gw_mtxel_project -- out[p][b] = sum_G M[p][G] sqrt(v(G)) U[G][b] (device out
 *   complex double[npairs][nb]) for matrix elements of dtype (device
 *   [npairs][neps]); gw_chi0_accumulate on it with neps := nb gives
 *   chi_B(w) = U^H V^1/2 chi0(w) V^1/2 U.  GW_EINVAL for bad sizes or aliasing.
 * gw_epsinv_from_basis -- eps^-1(w) from chi_B (device complex double
 *   [nfreq][nb][nb]): epst^-1 ~= I + U ((I - chi_B)^-1 - I) U^H, eps^-1 =
 *   V^1/2 epst^-1 V^-1/2 (device out complex double[nfreq][neps][neps]).
 *   Allocates its own buffers and synchronises.  GW_EINVAL for bad sizes, NULL
 *   arrays, aliasing, vcoul <= 0; GW_ESINGULAR from the small inverses.
 */
gw_status gw_lowrank_basis(gw_ctx* ctx, int neps, const double* chi0_static,
                           const double* vcoul, int nb, double* basis, double* eigenvalues);
gw_status gw_mtxel_project(gw_ctx* ctx, int npairs, int neps, const void* mtxel, gw_dtype dtype,
                           const double* vcoul, int nb, const double* basis, double* out);
gw_status gw_epsinv_from_basis(gw_ctx* ctx, int neps, int nb, int nfreq, const double* chi_b,
                               const double* vcoul, const double* basis, double* epsinv);

/*
 * gw_screened_w -- W_f[G][G'] = epsinv_f[G][G'] v(q+G') (Sec. II).
 *   epsinv (device) complex double[nfreq][neps][neps]; vcoul (device) double[neps];
 *   w      (device) out complex double[nfreq][neps][neps] (may be epsinv: in place).
 * Errors: GW_EINVAL for negative sizes, NULL arrays, nfreq > 65535.
 */
gw_status gw_screened_w(gw_ctx* ctx, int neps, int nfreq, const double* epsinv,
                        const double* vcoul, double* w);

/*
 * gw_sigma_sx -- the screened exchange with the static inverse dielectric matrix
 * (Sec. II, the SX term of the self-energy with its frequency argument at 0),
 * for one q, added to sigma:
 *   sigma[n] -= prefactor sum_{n''}^{occ} sum_{G,G'} conj(M_{n''n}(G)) M_{n''n}(G')
 *               epsinv[G][G'] v(q+G'),
 * computed as U = conj(M) epsinv on the matrix cores and per-band dot products
 * with v M, summed over n'' and G' in a fixed order.
 *   mtxel   (device) complex[nocc][nband][neps] of dtype: M_{n''n} at -q-G by the
 *           sphere index G (the caller's ordering, matching epsinv's).
 *   epsinv  (device) complex double[neps][neps] at omega = 0; vcoul (device) double[neps].
 *   prefactor  the q-point weight.
 *   sigma   (device) in/out complex double[nband]; may not alias an input.
 * Uses 2*nocc*nband*neps*16 bytes of context workspace.
 * Errors: GW_EINVAL for negative sizes, unknown dtype, NULL arrays, a non-finite
 * prefactor, nocc*nband > 65535, neps > 16384, or sigma aliasing an input.
 */
gw_status gw_sigma_sx(gw_ctx* ctx, int nocc, int nband, int neps, const void* mtxel,
                      gw_dtype dtype, const double* epsinv, const double* vcoul,
                      double prefactor, double* sigma);

/*
 * gw_unfold_spinor -- wavefunctions at k' = S k - G0 from those at k under a
 * space-group operation {S|tau}: r -> S r + tau (Sec. III, symmetries with spinor
 * wavefunctions, axis and angle extraction):
 *   cout[b][s][i] = sum_t U[s][t] cin[b][t][j] e^{-i G.tau},
 *   G = gout_i - G0 (the same plane wave relative to S k), gin_j = S^-1 G,
 * with the band-independent phase e^{-i S k.tau} dropped.  U is the SU(2) matrix
 * exp(-i theta/2 n.sigma) of the rotation part of S (S itself, or -S when
 * det S = -1: spin is unchanged by inversion), found from the quaternion of the
 * Cartesian rotation by Markley's form of Shepperd's method, positive branch.
 *   nspinor 1 or 2 (1: no spin rotation); nb bands.
 *   gin   (host) int[ng_in][3]  integer reciprocal coordinates of the sphere at k.
 *   cin   (device) complex[nb][nspinor][ng_in] of dtype.
 *   gout  (host) int[ng_out][3] the sphere at k' (any order).
 *   rot   (host) int[9] S in the lattice basis, row-major, acting on fractional
 *         coordinates of r (on integer reciprocal coordinates S acts as rot^-T).
 *   tau   (host) double[3] fractional translation in lattice coordinates.
 *   g0    (host) int[3] the reciprocal vector folding S k back, or NULL for 0.
 *   cell  (host) double[3] orthorhombic lattice constants (S_cart = A S A^-1).
 *   cout  (device) out complex[nb][nspinor][ng_out] of dtype; may not alias cin.
 * Arithmetic in double; c64 inputs are rounded once on output.  Synchronises the
 * context stream before returning (the index tables are staged from the host).
 * Errors: GW_EINVAL for nspinor not 1 or 2, negative sizes, unknown dtype, NULL
 * arrays, nb > 524280, det rot not +-1, rot not orthogonal in this cell,
 * duplicate or out-of-range input G, an output G whose preimage is not in gin,
 * cout aliasing cin.
 */
gw_status gw_unfold_spinor(gw_ctx* ctx, int nspinor, int nb, int ng_in, const int* gin,
                           const void* cin, gw_dtype dtype, int ng_out, const int* gout,
                           const int* rot, const double* tau, const int* g0,
                           const double* cell, void* cout);

/*
 * gw_chi0_symmetrize -- chi0(q) averaged over operations of the little group of q
 * (Sec. III: k-sums are unfolded with the little group of q).  For {S|tau} with
 * S q = q + G_S, the pair at S k has M_{Sk}(G) = e^{i(q+G).tau} M_k(S^-1 (G - G_S)), so
 *   chi_out[f][G][G'] = (1/nops) sum_S e^{-i(G-G').tau} chi_in[f][S^-1(G-G_S)][S^-1(G'-G_S)].
 * chi0 summed over the irreducible points of the little group, each weighted by
 * its orbit size, then passed through this call equals the full-grid sum.
 *   geps (host) int[neps][3] the eps sphere at q (closed under every operation).
 *   qred (host) double[3]; nops 1..96; rots (host) int[nops][9] S in the lattice
 *   basis, row-major, as for gw_unfold_spinor; taus (host) double[nops][3].
 *   chi_in (device) complex double[nfreq][neps][neps]; chi_out (device) out, same
 *   shape, not chi_in.
 * Synchronises the context stream (its tables are staged from the host).
 * Errors: GW_EINVAL for negative sizes, nops outside 1..96, NULL arguments,
 * aliasing, det S not +-1, an operation outside the little group of q, a sphere
 * not closed under an operation, duplicate G.
 */
/*
 * gw_little_group -- host bookkeeping, no context and no device work: which of
 * nops operations (rots as for gw_unfold_spinor) keep q, S q = q + G_S (Sec. III,
 * the little group of q).  in_group[s] = 1 or 0; gshift[s][3] = G_S (0 when not
 * in the group).  GW_EINVAL for NULL arrays or det S not +-1.
 */
gw_status gw_little_group(int nops, const int* rots, const double* qred, int* in_group,
                          int* gshift);

/*
 * gw_kgrid_orbits -- host bookkeeping, no context and no device work: orbits of
 * the unshifted grid k = (i1/n1, i2/n2, i3/n3), point index (i1 n2 + i2) n3 + i3,
 * under nops operations (normally the little group of q).  For every point i:
 * rep[i] the index of its orbit's first point, op[i] an operation with
 * S k_rep = k_i + G0, g0[i][3] that G0; weight[i] the orbit size at
 * representatives and 0 elsewhere; *nirr the number of orbits.  The k-sum over
 * the grid is then sum over representatives of weight * (its term), averaged
 * over the group by gw_chi0_symmetrize.  GW_EINVAL for non-positive sizes, more
 * than 2^26 points, NULL arrays, det S not +-1, or a grid not closed under an
 * operation.  Arrays: rep, op, weight int[n1 n2 n3]; g0 int[n1 n2 n3][3].
 */
gw_status gw_kgrid_orbits(int n1, int n2, int n3, int nops, const int* rots, int* rep, int* op,
                          int* g0, int* weight, int* nirr);

gw_status gw_chi0_symmetrize(gw_ctx* ctx, int neps, int nfreq, const int* geps,
                             const double* qred, int nops, const int* rots, const double* taus,
                             const double* chi_in, double* chi_out);

/*
 * gw_gpp_modes -- Hybertsen-Louie generalized plasmon-pole parameters of the
 * static eps^-1 (the model Sec. II and the computational details use for Sigma):
 *   Omega^2_GG' = wp^2 (q+G).(q+G') / |q+G|^2 rho(G-G') / rho(0),  wp^2 = 4 pi rho(0),
 *   wt^2_GG'    = Omega^2_GG' / (delta_GG' - eps^-1_GG'(q; 0)),  wt its principal root,
 * returned as amp = Omega^2 / wt and wtilde = wt.  A mode with |delta - eps^-1|
 * <= 1e-10 or Re wt^2 <= 0 has no pole: amp = 0, wtilde = 1.
 *   geps  (host) int[neps][3]; cell (host) double[3] orthorhombic lattice
 *         constants; qred (host) double[3] q in reduced coordinates (q + G != 0).
 *   box   (host) int[3] the grid of rho; each box[a] > 2 max |geps[.][a]|.
 *   rho   (device) complex double[box0][box1][box2]: the valence density's
 *         Fourier components at g mod box (rho(0) = electrons per bohr^3 > 0).
 *   epsinv (device) complex double[neps][neps] at omega = 0.
 *   amp, wtilde (device) out complex double[neps][neps], distinct from epsinv.
 * Synchronises the context stream (reads rho(0); stages q + G from the host).
 * Errors: GW_EINVAL for NULL arguments, neps > 46340, a non-positive cell or box,
 * q + G = 0, a box too small for G - G', rho(0) <= 0, overlapping outputs.
 */
gw_status gw_gpp_modes(gw_ctx* ctx, int neps, const int* geps, const double* cell,
                       const double* qred, const int* box, const double* rho,
                       const double* epsinv, double* amp, double* wtilde);

/*
 * gw_sigma_gpp -- diagonal SX and COH self-energy matrix elements for one q with
 * the plasmon-pole eps^-1 (Sec. II, the SX and COH terms), added to the outputs:
 *   sigma_sx[n][e]  -= prefactor sum_{n'' < nocc} m^H [(delta + Omega^2/(d^2 - wt^2)) v] m
 *   sigma_coh[n][e] += prefactor sum_{n'' < nn}  m^H [Omega^2 / (2 wt (d - wt)) v] m
 * with m = M_{n''n}, d = energies[n][e] - en[n''], v = v(q+G').  The COH term is
 * the w' > 0 integral of the pole's spectral weight, with v(q+G') as in SX.
 *   mtxel   (device) complex[nn][nband][neps] of dtype: M_{n''n}(G), the first
 *           nocc of the nn states n'' occupied.
 *   en      (device) double[nn] energies of the states n'' (Hartree).
 *   vcoul   (device) double[neps]; amp, wtilde (device) from gw_gpp_modes.
 *   nenergy 1..4 evaluation energies per band; energies (device) double[nband][nenergy].
 *   sigma_sx, sigma_coh (device) in/out complex double[nband][nenergy], distinct.
 * Each band's sums run in a fixed order (no atomics).  FP64 throughout; c64
 * matrix elements are widened.  Uses up to 256 MiB of context workspace.
 * Errors: GW_EINVAL for negative sizes, nocc > nn, unknown dtype, nenergy outside
 * 1..4, a non-finite prefactor, NULL arrays, neps > 46340, sigma_sx == sigma_coh.
 */
gw_status gw_sigma_gpp(gw_ctx* ctx, int nn, int nocc, int nband, int neps, const void* mtxel,
                       gw_dtype dtype, const double* en, const double* vcoul, const double* amp,
                       const double* wtilde, int nenergy, const double* energies,
                       double prefactor, double* sigma_sx, double* sigma_coh);

/*
 * gw_bse_kernel -- exchange and direct kernels of the Bethe-Salpeter equation in
 * the Tamm-Dancoff form for one k-point (Sec. II, K^X and K^D, whose spin
 * dependence is the spin trace inside M_nn'):
 *   kx[(v,c)][(v',c')] =  sum_G     conj(M_vc(G)) vx(G) M_v'c'(G)
 *   kd[(v,c)][(v',c')] = -sum_{G,G'} conj(M_cc'(G)) W_GG' M_vv'(G')
 * with pair index v*nc + c.  Exchange is repulsive and the screened direct term
 * attractive; the -i and i of the Green's-function form are absorbed.
 *   mvc (device) complex[nv][nc][neps], mcc [nc][nc][neps], mvv [nv][nv][neps]
 *       of dtype, as gw_mtxel_spinor writes them (left set, right set, G).
 *   vx  (device) double[neps] the bare Coulomb potential, its long-range G = 0
 *       entry set to 0 by the caller.
 *   w   (device) complex double[neps][neps] the screened interaction W = eps^-1 v.
 *   kx, kd (device) out complex double[nv*nc][nv*nc], overwritten; distinct, and
 *       neither may alias an input.
 * FP64 matrix-core GEMMs; c64 inputs are widened.  Uses about
 * 16 (2 nv nc N + 2 nc^2 N + nv^2 N + nc^2 nv^2) bytes of context workspace.
 * Errors: GW_EINVAL for negative sizes, unknown dtype, NULL arrays, aliasing,
 * nv*nc or neps above 46340; GW_ENOMEM if the workspace cannot be allocated.
 */
gw_status gw_bse_kernel(gw_ctx* ctx, int nv, int nc, int neps, const void* mvc, const void* mcc,
                        const void* mvv, gw_dtype dtype, const double* vx, const double* w,
                        double* kx, double* kd);

/*
 * gw_peak_probe -- measured peak of the device, to set beside the nominal
 * roofline figures: kind 0 an FP64 matrix-core loop (TFLOP/s, v_mfma 16x16x4
 * FP64, eight independent chains per wavefront), kind 1 an FP64 vector FMA loop
 * (TFLOP/s), kind 2 a 1 GiB device-to-device copy (GB/s, bytes read + written).
 * Best of three timed runs after one warm-up; synchronises.  Allocates 8 MiB
 * (and 2 GiB for kind 2) for the duration of the call.
 * Errors: GW_EINVAL for a NULL result or another kind; GW_ENOMEM.
 */
gw_status gw_peak_probe(gw_ctx* ctx, int kind, double* result);

/* ------------------------------------------------------------------------ */
/* Learned closure of the truncated conduction-band sum.                      */
/* ------------------------------------------------------------------------ */
typedef struct gw_mlp gw_mlp;

typedef enum {
  GW_CLOSURE_INFER = 0,         /* chi0_out = chi0_trunc + Hermitised network remainder */
  GW_CLOSURE_TRAIN_STEP = 1,    /* one Adam step on the MSE to (chi0_full - chi0_trunc) */
  GW_CLOSURE_FULL_FALLBACK = 2  /* chi0_out = chi0_full (the full band sum) */
} gw_closure_mode;

/* Network: nin -> depth hidden layers of `width` (SiLU) -> nout, weights
 * initialised from `seed`.  bf16 matrix-core products, float master weights. */
gw_status gw_mlp_create(gw_ctx* ctx, gw_mlp** net, int nin, int width, int depth,
                        int nout, uint64_t seed);
gw_status gw_mlp_destroy(gw_mlp* net);
/* Serialise float master weights and Adam state to a host buffer.  Call with
 * host_buf = NULL to query *nbytes. */
gw_status gw_mlp_save(const gw_mlp* net, void* host_buf, size_t* nbytes);
gw_status gw_mlp_load(gw_mlp* net, const void* host_buf, size_t nbytes);
/* Largest rel_F against the full sum at which gw_chi0_closure keeps a
 * prediction (INFER with chi0_full); default 1e-4.  GW_EINVAL if tol < 0 or
 * non-finite. */
gw_status gw_mlp_set_tolerance(gw_mlp* net, double tol);

/*
 * gw_chi0_closure -- predict the remainder chi0_full - chi0_trunc of one
 * (q, omega = 0) matrix from per-(G,G') features (G <= G' only):
 *   |q+G|, |q+G'|, (q+G).(q+G')... see the design notes for the exact list:
 *   |q+G|, |q+G'|, G.G' (Cartesian), Re chi0_trunc, Im chi0_trunc, gap, emax.
 *   qG          (device) double[neps][3] Cartesian q+G.
 *   chi0_trunc  (device) complex double[neps][neps].
 *   chi0_full   (device) complex double[neps][neps]: training target
 *               (TRAIN_STEP) or the fallback value (FULL_FALLBACK / fallback check).
 *   lr          Adam learning rate (TRAIN_STEP).
 *   loss        (host) out float: the MSE before the step, or NULL.
 *   chi0_out    (device) out complex double[neps][neps] (INFER, FULL_FALLBACK).
 * In INFER mode with chi0_full given, the full sum judges the prediction:
 * rel_F = ||chi0_out - chi0_full||_F / ||chi0_full||_F is reduced on the device
 * in a fixed order, and if it exceeds the network's tolerance
 * (gw_mlp_set_tolerance, default 1e-4) or the corrected matrix is not negative
 * semidefinite (a double-precision Cholesky of -chi0_out fails), the full sum is
 * written instead and GW_EFALLBACK is returned.  That check synchronises the
 * context stream.  Without chi0_full the prediction is returned unjudged.
 */
gw_status gw_chi0_closure(gw_ctx* ctx, gw_mlp* net, int mode, int neps,
                          const double* qG, const double* chi0_trunc, double gap,
                          double emax, const double* chi0_full, float lr, float* loss,
                          double* chi0_out);

/* ------------------------------------------------------------------------ */
/* Batched many-q plan: one captured graph over every q.                      */
/* ------------------------------------------------------------------------ */
typedef struct gw_plan gw_plan;

/* Per-q description (host struct; the pointers it holds are device pointers
 * except gv/gc/geps, which are host). */
typedef struct {
  int nv, ngv;  const int32_t* gv;  const void* cv;    /* valence at k+q */
  int nc, ngc;  const int32_t* gc;  const void* cc;    /* conduction at k */
  int neps;     const int32_t* geps;
  const double* ev;  const double* ec;                 /* (device) energies */
  const double* vcoul;                                 /* (device) v(q+G) */
  int head_index;                                      /* G = 0 index or -1 */
  double* chi0;                                        /* (device) out [nfreq][neps][neps] */
  double* epsinv;                                      /* (device) out [nfreq][neps][neps] */
} gw_q_desc;

/* All q share box, nspinor, dtype, precision and frequencies. */
gw_status gw_plan_create(gw_ctx* ctx, gw_plan** plan, const int box[3], int nspinor,
                         gw_dtype dtype, gw_prec prec, int nfreq, const double* omega,
                         double prefactor, int nq, const gw_q_desc* q);
/* Autotune tile shapes (timed trial launches) and capture every stage of every
 * q into one HIP graph.  Allocates all workspace. */
gw_status gw_plan_compile(gw_plan* plan);
/* Replay the graph on the context stream; synchronises and reports
 * GW_ESINGULAR if any q's eps had a zero pivot. */
gw_status gw_plan_launch(gw_plan* plan);
gw_status gw_plan_destroy(gw_plan* plan);
/* Autotuner result for the plan as a short text (valid until the plan is destroyed). */
const char* gw_plan_describe(const gw_plan* plan);

#ifdef __cplusplus
}
#endif
#endif /* GW_SPINOR_H */

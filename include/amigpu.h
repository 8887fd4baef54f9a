/*
 * amigpu -- batched algorithmic Matsubara integration (AMI) on MI355X (gfx950).
 *
 * C ABI of libamigpu.so.  The method is that of Burke & LeBlanc, "TorchAmi:
 * Generalized CPU/GPU Implementation of Algorithmic Matsubara Integration"
 * (arXiv 2311.17189):
 *
 *   construct: the integrand of Eq. (1), a product of propagators Eq. (2)
 *              G_j = 1 / (sum_l alpha_jl w_l + sum_i eps_ji E_i), is summed over
 *              the fermionic Matsubara frequencies nu_1..nu_n (w_l = i nu_l) by
 *              repeated residues (Eqs. (3)-(4)), giving terms A * FT * R (Eq. (6));
 *   evaluate:  the terms are evaluated for a batch of N_E energy rows and N_F
 *              external-frequency rows, giving an [N_F, N_E] result (Sec. 2.3).
 *
 * Conventions shared by every call:
 *   - Integers labelling a diagram are row-major int8.  Frequency slot order is
 *     the summed frequencies first, external frequencies last (Sec. 5.1.1).
 *   - Complex values are interleaved (re, im) float64 pairs (complex128).
 *   - Buffers passed to evaluate calls are DEVICE pointers on the device that is
 *     current on the calling thread; the caller owns them.  Scalars and arrays
 *     documented as host arrays are read before the call returns.
 *   - Evaluate calls are asynchronous on `hip_stream` (a hipStream_t; NULL is the
 *     default stream).  All argument checks happen on the host before any launch;
 *     a non-AMI_OK status means nothing was launched.  The message of the last
 *     failure on the calling thread is returned by amiLastError().
 *   - An AmiTerms handle may be used from several threads for evaluation once it
 *     has been uploaded to a device (amiTermsUpload); construction and amiFree
 *     must not race with other uses of the same handle.
 */
#ifndef AMIGPU_H
#define AMIGPU_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    AMI_OK = 0,
    AMI_E_ARG = -1,         /* bad pointer, size, stride or flag                  */
    AMI_E_LABEL = -2,       /* invalid labels (see amiConstruct)                   */
    AMI_E_MULTIPOLE = -3,   /* two denominators share a pole (Eq. (5) not handled) */
    AMI_E_COEFF = -4,       /* summed frequency with coefficient other than +-1    */
    AMI_E_HIP = -5,         /* a HIP runtime call failed                           */
    AMI_E_OOM = -6,         /* allocation failed                                   */
    AMI_E_UNSUPPORTED = -7  /* valid input outside what this build evaluates       */
} AmiStatus;

/* amiConstruct flags */
#define AMI_FACTORIZE 1u    /* also build the factorized Fermi tree (Sec. 2.1, Fig. 1) */
#define AMI_MULTIPOLE 2u    /* take poles of higher order by Eq. (5) instead of failing */

typedef struct AmiTerms AmiTerms;

/*
 * amiConstruct -- symbolic solution of one integrand (Sec. 2.2; Sec. 5.1.2).
 *
 *   n_g       number of propagators in R0 (rows), >= 1
 *   n_eps     length of each epsilon_t row (energy placeholders), 1..32
 *   n_freq    length of each alpha_t row (summed + external frequencies), 1..16
 *   n_int     number of nested sums, 0..n_freq; slots 0..n_int-1 are summed in order
 *   alpha     host int8 [n_g][n_freq], entries in {-1,0,1}
 *   eps       host int8 [n_g][n_eps],  entries in {-1,0,1}
 *   fermionic host uint8 [n_freq]: nonzero = fermionic frequency; NULL = all
 *             fermionic.  Summed slots must be fermionic (Eq. (3)).
 *   flags     0, AMI_FACTORIZE or AMI_MULTIPOLE (not both).  With AMI_MULTIPOLE a
 *             pole shared by M denominators is taken by Eq. (5): the Leibniz rule
 *             over the pole's Fermi/Bose function and the other denominators gives
 *             terms whose leaves are Taylor coefficients T_j(x) = (1/j!) d^j/dx^j
 *             f(beta x) (leaf code sigma*(1+j)) and whose denominators carry powers
 *             (repeated entries); such solutions are evaluated by the specialized
 *             forward kernels only
 *   out       receives a new handle (owned by the caller, release with amiFree)
 *
 * Host-only: no device memory is touched.  Errors: AMI_E_ARG (sizes/pointers),
 * AMI_E_LABEL (coefficients outside {-1,0,1}, bosonic summed slot, a summed
 * frequency absent from every denominator of a term), AMI_E_COEFF (a summed
 * frequency reached coefficient +-2 through a substitution), AMI_E_MULTIPOLE
 * (coincident poles, or a denominator that vanishes identically).
 */
AmiStatus amiConstruct(int32_t n_g, int32_t n_eps, int32_t n_freq, int32_t n_int,
                       const int8_t *alpha, const int8_t *eps, const uint8_t *fermionic,
                       uint32_t flags, AmiTerms **out);

/* Release a handle and its device tables (every device it was uploaded to). */
void amiFree(AmiTerms *terms);

/*
 * Feynman-graph input (Sec. 2.5).  A graph is a list of lines, 4 integers each:
 * source vertex, target vertex, B/F (0 bosonic, 1 fermionic), spin (carried,
 * unused).  Fermionic lines point along the fermion flow, which is also the
 * direction of their frequency and momentum.
 *
 * amiReadGraph -- parse the plain-text form (one line per row, whitespace
 * separated, '#' starts a comment) into edges (host int32 [cap][4]); *n_edges
 * and *n_vertices (1 + the largest vertex index) are set even when edges is
 * NULL.  AMI_E_ARG on unreadable files, malformed rows or a small buffer.
 */
AmiStatus amiReadGraph(const char *path, int32_t *edges, int32_t cap, int32_t *n_edges, int32_t *n_vertices);

/*
 * amiConstructGraph -- momentum-conserving labels for a graph and the
 * construction of its integrand (amiConstruct with R0 = the labels of the
 * fermionic lines, in edge order, and one energy per fermionic line).
 * The external frequency enters at the vertex without an incoming fermionic
 * line and leaves at the one without an outgoing one (self-energy legs, a
 * fermionic external slot); with no such vertices, at the two vertices
 * without a bosonic line (a bosonic external slot).  A spanning tree is grown
 * from the bosonic lines first, then the fermionic ones, in edge order; each
 * line outside it carries one summed frequency (slots in edge order) flowing
 * source -> target on it and back through the tree; the external frequency
 * flows along the tree path between the external vertices.  Every vertex may
 * have at most one fermionic line in and one out.  Errors: AMI_E_ARG (sizes,
 * ranges), AMI_E_LABEL (unbalanced or disconnected graphs, no external legs,
 * a summed frequency on a bosonic line, and amiConstruct's), AMI_E_UNSUPPORTED
 * (more than 15 loops or 32 propagators).  amiTermsLabels returns the labels.
 */
AmiStatus amiConstructGraph(int32_t n_vertices, int32_t n_edges, const int32_t *edges, uint32_t flags,
                            AmiTerms **out);

/* R0 of a handle: alpha [n_g][n_freq], eps [n_g][n_eps], fermionic [n_freq]
 * (host buffers sized from amiTermsInfo; any may be NULL). */
AmiStatus amiTermsLabels(const AmiTerms *terms, int8_t *alpha, int8_t *eps, uint8_t *fermionic);

/*
 * amiTermsInfo -- sizes of the solution, info[0..15] (host array):
 *   0 T       flat terms after canonical merging (FACTORIZE=false form, Sec. 2.2)
 *   1 n_int   2 n_eps   3 n_freq   4 n_ext (= n_freq - n_int)
 *   5 L       distinct leaves (Fermi/Bose functions of an energy combination)
 *   6 D       distinct denominators
 *   7 G       groups of terms sharing the same denominators (the top level of
 *             the factorized form: FT_g * R_g)
 *   8 tree nodes of the factorized Fermi tree (0 unless built with AMI_FACTORIZE)
 *   9 raw terms before canonical merging
 *   10 leaves per term (= n_int)   11 denominators per term (= n_g - n_int;
 *      the most a term holds when info[15] is 0)
 *   12 packed form available (1/0)   13 the packed kernels build Fermi leaves
 *      from products of exp(beta E_i) (1/0)
 *   14 n_g (propagators of R0)
 *   15 uniform (1): plain leaves and n_g - n_int denominators in every term;
 *      0 after poles of higher order (AMI_MULTIPOLE)
 */
AmiStatus amiTermsInfo(const AmiTerms *terms, int64_t info[16]);

/*
 * amiTermsCanonical -- the canonical flat term list as an int32 stream:
 *   header n_int, n_eps, n_freq, T; then per term: prefactor s; n_int leaves as
 *   (sigma, e[0..n_eps)); (n_g - n_int) denominators as (e[0..n_eps), a[0..n_freq)).
 *   With poles of higher order (AMI_MULTIPOLE) a leaf's first entry is the code
 *   sigma*(1+j) of its Taylor coefficient, and when the terms do not all hold the
 *   same number of denominators the header holds -T and each term's s is
 *   followed by its number of denominators (repeated entries are powers).
 * sigma = +1 is the Fermi function 1/(exp(y)+1), -1 is 1/(1-exp(y)) (= -n_B).
 * Canonical: each denominator's first non-zero coefficient is positive (its sign
 * moved into s), leaves sorted by (sigma, e), denominators by (e, a), equal
 * terms merged, terms sorted by (leaves, denominators).
 * With `from_tree` nonzero the list is the expansion of the factorized tree
 * (requires AMI_FACTORIZE).  If buf is NULL or cap is too small, *len gets the
 * required length and AMI_E_ARG is returned when buf is non-NULL.
 */
AmiStatus amiTermsCanonical(const AmiTerms *terms, int32_t from_tree, int32_t *buf,
                            int64_t cap, int64_t *len);

/* Upload the evaluation tables to the current device (done on first evaluate
 * otherwise; call it before capturing evaluate calls into a HIP graph). */
AmiStatus amiTermsUpload(AmiTerms *terms);

/*
 * amiEvaluate -- batched evaluation (Sec. 2.3):
 *   out[f][s] = sum_t s_t * prod_leaves f_sigma(beta*(e.E_s) [+ beta*e_reg if sigma=-1])
 *                          / prod_dens (e.E_s + a_ext . w_f)
 *
 *   energies   device float64, element (s, i) at energies[s*stride_s + i*stride_i],
 *              s < n_e, i < n_eps.  (The paper's energy_t [N_E][N] is stride_s =
 *              n_eps, stride_i = 1.)  Real energies.
 *   n_e        energy rows (>= 0; 0 launches nothing but still zeroes out_sum)
 *   ext_freqs  device complex128 [n_f][n_ext]: the external slots of frequency_t
 *              (i nu for Matsubara, omega + i Gamma for real frequency, Sec. 1)
 *   n_f        frequency rows (>= 1)
 *   beta       inverse temperature (> 0); e_reg regulator added to the energy
 *              argument of Bose-type leaves only (0 disables it)
 *   out        device complex128 [n_f][n_e], or NULL
 *   out_sum    device complex128 [n_f] = sum over s of out[f][s] (the Monte-Carlo
 *              row sum of Sec. 2.3), or NULL.  Reduced in a fixed order: repeated
 *              calls give bitwise-equal results.
 * At least one of out/out_sum must be non-NULL.  The per-block partial sums go
 * to a workspace the handle keeps per device and stream (allocated on the first
 * call on a stream, grown on demand, released by amiFree): once a call on a
 * stream has sized it, later calls of that size allocate nothing and may be
 * captured in a HIP graph.  Calls on different streams use different
 * workspaces; the adjoint entry points share the same ones.
 */
AmiStatus amiEvaluate(AmiTerms *terms,
                      const double *energies, int64_t n_e, int64_t stride_s, int64_t stride_i,
                      const double *ext_freqs, int64_t n_f,
                      double beta, double e_reg,
                      double *out, double *out_sum, void *hip_stream);

/*
 * amiEvaluateHubbard -- amiEvaluate with the energies computed in the kernel
 * from momenta (Sec. 5.2): K_j = sum_l alpha_jl k_l with the external momentum
 * q in the external slot, E_j = -eps(K_j) = 2t(cos K_jx + cos K_jy) + mu (2D
 * square lattice).  Requires n_eps == n_g (one energy per propagator).
 *
 *   k        device float64 [n_e][2*n_int] row-major (k1x k1y k2x k2y ...),
 *            row stride stride_k (>= 2*n_int) in doubles.  Components are
 *            reduced modulo 2 pi in the kernel (exact for |k| < 6e6; the
 *            dispersion is 2 pi periodic)
 *   q        host float64 [2*n_ext]
 */
AmiStatus amiEvaluateHubbard(AmiTerms *terms,
                             const double *k, int64_t n_e, int64_t stride_k,
                             const double *q, double t, double mu,
                             const double *ext_freqs, int64_t n_f,
                             double beta, double e_reg,
                             double *out, double *out_sum, void *hip_stream);

/*
 * amiEvaluateComplex -- amiEvaluate at complex energies (the energy vector's
 * element type is complex, Sec. 5.1.3; e.g. energies with a broadening):
 *
 *   energies  device complex128 [n_e][n_eps] as interleaved (re, im) doubles;
 *             element (s, i) at energies[2*(s*stride_s + i*stride_i)], the
 *             strides counted in complex elements (>= 1)
 *
 * Every other argument, the output layout and the ownership are those of
 * amiEvaluate.  The leaves f(beta x) and the denominators are taken at the
 * complex x = e . E (the analytic continuation of the real-energy result);
 * the regulator e_reg shifts the real part of Bose-type leaf arguments.
 * Leaves are accurate for |beta Im x| < 6e6; a Fermi leaf has poles at
 * beta x = i pi (2n+1), which the caller keeps away from.  Served by the
 * specialized kernels only (compiled on first use, as AMI_VARIANT_SPECIALIZED):
 * in one pass up to 1024 terms; in two passes (the complex group sums and
 * energies stored per sample in the chunked workspace of AMI_VARIANT_TWO_PASS,
 * then evaluated per frequency row; at most 65535 rows) above, up to 4096
 * terms, or at any size when the handle's variant is AMI_VARIANT_TWO_PASS.
 * AMI_E_UNSUPPORTED for solutions outside their form and for poles of higher
 * order (AMI_MULTIPOLE).  Its adjoint is amiEvaluateComplexAdjoint.
 */
AmiStatus amiEvaluateComplex(AmiTerms *terms,
                             const double *energies, int64_t n_e, int64_t stride_s, int64_t stride_i,
                             const double *ext_freqs, int64_t n_f,
                             double beta, double e_reg,
                             double *out, double *out_sum, void *hip_stream);

/*
 * amiEvaluateComplexAdjoint -- reverse-mode derivatives of amiEvaluateComplex
 * (Sec. 5.1.3: complex energies).  The result is analytic in every energy, so
 * for the real objective L = Re sum_{f,s} conj(c[f][s]) out[f][s], with
 * c[f][s] = grad_out[f][s] + grad_sum[f] (either may be NULL, not both), it
 * returns
 *   grad_energies complex [n_e][n_eps] row-major, interleaved (device, or
 *                 NULL): dL/dRe E + i dL/dIm E = sum_f c[f][s] conj(dI/dE),
 *                 the convention of grad_freqs; at real energies its real
 *                 part is amiEvaluateAdjoint's grad_energies
 *   grad_beta     [1]: dL/dbeta (real; device, or NULL)
 *   grad_freqs    complex [n_f][n_ext]: as amiEvaluateAdjoint (device, or NULL)
 * using f_sigma'(y) = -f_sigma(y) f_sigma(-y) at complex y and
 * d(1/D)/dD = -1/D^2.  energies, strides, ext_freqs, beta, e_reg: as
 * amiEvaluateComplex; out / out_sum (device, or NULL) receive the forward
 * values on the way.  The sums over samples are reduced in a fixed order.
 * Served by the specialized kernels (compiled on first use): one pass up to
 * 512 terms (up to 1024 under AMI_VARIANT_SPECIALIZED); above, or under
 * AMI_VARIANT_TWO_PASS, passes over the chunked workspace of the two-pass
 * variant (complex group sums and energies stored; per frequency row the
 * values and the complex cotangents of group sums and denominators; then the
 * leaves' complex cotangents by reverse sweeps), up to 4096 terms.
 * AMI_E_UNSUPPORTED for solutions outside their form and for poles of higher
 * order.
 */
AmiStatus amiEvaluateComplexAdjoint(AmiTerms *terms,
                                    const double *energies, int64_t n_e, int64_t stride_s, int64_t stride_i,
                                    const double *ext_freqs, int64_t n_f,
                                    double beta, double e_reg,
                                    const double *grad_out, const double *grad_sum,
                                    double *grad_energies, double *grad_beta, double *grad_freqs,
                                    double *out, double *out_sum, void *hip_stream);

/*
 * amiEvaluateAdjoint -- reverse-mode derivatives of the batched evaluation.
 * For the real objective L = Re sum_{f,s} conj(c[f][s]) out[f][s] with the
 * cotangent c[f][s] = grad_out[f][s] + grad_sum[f] (either may be NULL, not
 * both; grad_sum is the cotangent of out_sum), it returns
 *   grad_energies [n_e][n_eps] row-major: dL/dE (device, or NULL)
 *   grad_beta     [1]: dL/dbeta at fixed frequency values (device, or NULL)
 *   grad_freqs    complex [n_f][n_ext]: conj(dL/dw) summed over samples, the
 *                 gradient of a real loss with respect to a complex input
 *                 (d/dRe w + i d/dIm w) (device, or NULL)
 * using d f_sigma/dy = -f_sigma (1 - f_sigma) for every leaf and
 * d(1/D)/dD = -1/D^2 for every denominator (the terms of Eq. (6) are products
 * of these); a Taylor-coefficient leaf of a pole of higher order (Eq. (5)),
 * T_j(x) = beta^j f^(j)(beta x) / j!, has dT_j/dx = (j + 1) T_(j+1) and
 * dT_j/dbeta = (j T_j + x dT_j/dx) / beta.  Other arguments as amiEvaluate.
 * The sums over samples are reduced in a fixed order.  Served by the
 * specialized kernels (in one pass up to 128 terms, in passes up to 4096; see
 * the variants below; poles of higher order only there) or by the packed ones
 * (every energy coefficient +-1, at most 255 distinct leaves and
 * denominators, at most 8 of each per term, no leaf twice in one term):
 * AMI_E_UNSUPPORTED when none applies.
 * out / out_sum (device, or NULL): the forward values, as amiEvaluate would
 * return them (up to rounding when the adjoint runs in passes), computed on
 * the way -- a value-and-gradient pass when the cotangents do not depend on
 * the values (e.g. grad_sum for a Monte-Carlo estimate).
 */
AmiStatus amiEvaluateAdjoint(AmiTerms *terms,
                             const double *energies, int64_t n_e, int64_t stride_s, int64_t stride_i,
                             const double *ext_freqs, int64_t n_f, double beta, double e_reg,
                             const double *grad_out, const double *grad_sum,
                             double *grad_energies, double *grad_beta, double *grad_freqs,
                             double *out, double *out_sum, void *hip_stream);

/*
 * amiEvaluateHubbardAdjoint -- the adjoint of amiEvaluateHubbard: as
 * amiEvaluateAdjoint, with the energies' cotangent carried to the momenta
 * through dE_j/dK_jc = -2t sin K_jc and K_j = sum_l alpha_jl k_l (Sec. 5.2):
 *   grad_k  [n_e][2*n_int] row-major, dL/dk (device, or NULL)
 *   grad_mu, grad_t  [1] each: dL/dmu, dL/dt summed over samples (device, or NULL)
 */
AmiStatus amiEvaluateHubbardAdjoint(AmiTerms *terms,
                                    const double *k, int64_t n_e, int64_t stride_k,
                                    const double *q, double t, double mu,
                                    const double *ext_freqs, int64_t n_f,
                                    double beta, double e_reg,
                                    const double *grad_out, const double *grad_sum,
                                    double *grad_k, double *grad_mu, double *grad_t,
                                    double *grad_beta, double *grad_freqs,
                                    double *out, double *out_sum, void *hip_stream);

/*
 * amiEvaluateHubbardAdjointNoAlloc -- amiEvaluateHubbardAdjoint for callers
 * that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  Same arguments, layouts,
 * kernels and results (bit for bit) as amiEvaluateHubbardAdjoint; it calls no
 * hipMalloc, hipFree or other allocating routine:
 *   - the partial sums over samples go to a scratch array of
 *     AMI_NOALLOC_SCRATCH_BYTES inside the library (one per device, held until
 *     the process ends; its address is looked up on the first call on a
 *     device).  Calls that need more -- about (4 + 2 n_f n_ext + 2 n_f) * 8 / 64
 *     bytes per sample, i.e. n_e up to about 16.7 million at n_f = 1 -- fail
 *     with AMI_E_ARG: split the samples;
 *   - the handle's tables must already be on the current device
 *     (amiTermsUpload, or an earlier evaluate call), else AMI_E_ARG;
 *   - when the call is served by a specialized kernel, that kernel must
 *     already be loaded on the current device (amiTermsSpecialize(terms, 1) with
 *     the device current, or an earlier amiEvaluateHubbardAdjoint call), else
 *     AMI_E_ARG; nothing is compiled or loaded.
 * Every call on one device shares that device's scratch: calls that overlap
 * on one device (two streams, two threads) race and give wrong sums; the
 * scratch keeps the last call's partial sums, every one of which a call
 * writes before reading it.
 */
#define AMI_NOALLOC_SCRATCH_BYTES (16u << 20)
AmiStatus amiEvaluateHubbardAdjointNoAlloc(AmiTerms *terms,
                                           const double *k, int64_t n_e, int64_t stride_k,
                                           const double *q, double t, double mu,
                                           const double *ext_freqs, int64_t n_f,
                                           double beta, double e_reg,
                                           const double *grad_out, const double *grad_sum,
                                           double *grad_k, double *grad_mu, double *grad_t,
                                           double *grad_beta, double *grad_freqs,
                                           double *out, double *out_sum, void *hip_stream);

/*
 * amiIntegrateHubbard -- Monte-Carlo integration of the integrand over the
 * internal momenta (Sec. 5.2; the row average of Sec. 2.3), sampling in the
 * kernel: sample s (0 <= s < n_samples) draws its 2*n_int momentum
 * components, row-major as the k rows of amiEvaluateHubbard, from Philox4x32
 * with 10 rounds (Salmon et al., SC'11): the words of the blocks with counter
 * (s mod 2^32, s div 2^32, b, 0), b = 0, 1, ..., and key (seed mod 2^32,
 * seed div 2^32), component c from word c as (u - 1/2) * 2 pi with
 * u = (word + 1/2) / 2^32, i.e. uniform on (-pi, pi).  No sample touches
 * device memory -- except for solutions AUTO evaluates in two passes (more
 * than 1024 terms, up to 4096, or 2 G + 4 D > 128): the first pass draws the
 * momenta and stores each sample's group sums and energies in the chunked
 * workspace, the second accumulates the sums per frequency row.
 *   q, t, mu      as amiEvaluateHubbard
 *   ext_freqs     device complex128 [n_f][n_ext], 1 <= n_f <= 8 (split longer lists)
 *   sums          device float64 [n_f][4]: sum over the samples of Re I, Im I,
 *                 (Re I)^2, (Im I)^2.  The estimate of the integral with measure
 *                 d^2k/(2 pi)^2 per loop is (sum Re I + i sum Im I) / n_samples;
 *                 the squares give its standard error.
 * The sums are reduced in a fixed order for a given device: repeated calls give
 * the same bits.  Needs the specialized kernels (AMI_E_UNSUPPORTED beyond
 * their limits, whatever the handle's variant); the kernels are compiled on
 * first use.  Uses the handle's per-stream workspace.
 */
AmiStatus amiIntegrateHubbard(AmiTerms *terms, int64_t n_samples, uint64_t seed,
                              const double *q, double t, double mu,
                              const double *ext_freqs, int64_t n_f, double beta, double e_reg,
                              double *sums, void *hip_stream);

/*
 * Kernel variants of a handle (amiSetVariant).  All evaluate the same
 * solution (Sec. 2.3); they differ in how the term tables reach the kernel:
 *   AMI_VARIANT_AUTO         (default) specialized when the solution has at
 *                            most 1024 flat terms (4096 in passes) and at
 *                            most 16 energies and its kernels compile -- the
 *                            forward in two passes (below) when the solution
 *                            has more than 1024 terms (up to 4096) or when its
 *                            groups and denominators would not fit the one-pass
 *                            kernel's registers (2 G + 4 D > 128), the adjoint
 *                            in passes (below) above 128 terms -- else
 *                            packed when the solution
 *                            has the packed form (+-1 coefficients, at most 255
 *                            leaves/denominators, 8 per term), else tables
 *   AMI_VARIANT_TABLES       one generic kernel over double-valued tables
 *                            (forward only, any coefficients; the per-diagram
 *                            baseline)
 *   AMI_VARIANT_PACKED       bit-mask tables read by kernels specialized per
 *                            self-energy shape
 *   AMI_VARIANT_SPECIALIZED  the diagram's own straight-line kernels, generated
 *                            from its tables and compiled at run time (hipRTC)
 *                            on first use -- or by amiTermsSpecialize -- and
 *                            cached on disk (AMIGPU_CACHE_DIR, else
 *                            $HOME/.cache/amigpu/jit); the forward in two
 *                            passes where AUTO would take them
 *   AMI_VARIANT_TWO_PASS     the specialized forward in two passes: a first
 *                            kernel stores every sample's group sums and
 *                            energies in a workspace (in chunks of at most
 *                            1 GiB), a second evaluates, per frequency row,
 *                            the denominators and the group products against
 *                            them; register use independent of the number of
 *                            groups; at most 65535 frequency rows per call.
 *                            The adjoint in passes over the same workspace
 *                            (per chunk of samples): that first kernel, then
 *                            one that per frequency row forms the values, the
 *                            group sums' cotangents and the denominators'
 *                            (stored), then one that forms the leaves'
 *                            cotangents by a reverse sweep of each group's
 *                            nested sum and finishes the gradients; its values
 *                            equal the forward's up to rounding
 * A forced variant that cannot serve a call fails it (AMI_E_UNSUPPORTED, or
 * AMI_E_HIP when the run-time compilation fails); AUTO falls back in the order
 * above and amiLastVariant names what ran and why.
 *
 * Tuning overrides of the generated kernels, read from the environment when a
 * kernel is generated (each changes the source, so the disk cache keeps the
 * forms apart): AMIGPU_JIT_ADJ_WAVES (one-pass adjoint's waves per SIMD floor,
 * default 2), AMIGPU_JIT_PARK_DV (0/1: the adjoint's leaf slopes in LDS),
 * AMIGPU_JIT_NESTED_COTANGENTS (terms per part of the one-pass adjoints'
 * nested leaf-cotangent sweep, 0 for per-term products; by default both forms
 * are compiled and the one whose code object spills no more and keeps the
 * occupancy is kept), AMIGPU_JIT_CADJ_PART and AMIGPU_JIT_CADJL_WAVES (terms
 * per part and waves floor of the complex adjoint's leaf pass, defaults 64
 * and 1).
 */
enum { AMI_VARIANT_AUTO = 0, AMI_VARIANT_TABLES = 1, AMI_VARIANT_PACKED = 2, AMI_VARIANT_SPECIALIZED = 3,
       AMI_VARIANT_TWO_PASS = 4 };

AmiStatus amiSetVariant(AmiTerms *terms, int32_t variant);

/*
 * amiSetTwoPassChunkBytes -- bound (bytes, >= 64 KiB; default 1 GiB) on the
 * workspace of one chunk of samples of the two-pass forward (real or complex
 * energies) and of the adjoint in passes, for every handle of the process: a
 * call with more samples than fit runs chunk after chunk.
 * Takes effect at the next call; the workspace never shrinks.
 */
AmiStatus amiSetTwoPassChunkBytes(int64_t bytes);

/*
 * amiTermsSpecialize -- compile (or load from the disk cache) the specialized
 * kernels of a handle for the energy (momentum = 0) or momentum (momentum = 1)
 * input and load them on the current device, so that the compilation stays
 * out of later evaluate calls.  Host-blocking.  AMI_E_UNSUPPORTED when the
 * solution is outside the specialized form, AMI_E_HIP when compiling or loading
 * fails (amiLastError holds the compiler log).  The kernels are the forward
 * (its two passes where AUTO takes them), the adjoint AUTO uses (one pass up
 * to 128 terms, its passes above), and for solutions of at most 1024 terms
 * the complex-energy forward and the kernels of its adjoint that AUTO uses
 * (amiEvaluateComplex, amiEvaluateComplexAdjoint) for the energy input, above
 * that the two passes of the complex-energy forward; all are compiled before a
 * device is touched.  A solution with Taylor-coefficient leaves (AMI_MULTIPOLE)
 * gets no complex-energy kernels.
 */
AmiStatus amiTermsSpecialize(AmiTerms *terms, int32_t momentum);

/*
 * amiTermsSource -- the generated device source of the specialized kernels
 * (energy input: momentum = 0; momentum input: 1; plus 2 for the source of the
 * two-pass forward, up to 4096 terms), NUL-terminated, into buf
 * (host, capacity cap bytes; *len receives the size including the NUL, also
 * when buf is NULL).  The source includes the library's device headers by
 * name (device_common.hpp, kargs.hpp, jit_kernel.hpp).  AMI_E_UNSUPPORTED when
 * the solution is outside the specialized form, AMI_E_ARG when cap is too small.
 */
AmiStatus amiTermsSource(const AmiTerms *terms, int32_t momentum, char *buf, int64_t cap, int64_t *len);

/*
 * amiBatchSource -- the generated device source of one module of the
 * persistent specialized batch (amiBatchCreate with tuning.kernels = 2) for
 * the n handles terms[0..n) with n_f[i] frequency rows each (host arrays;
 * momentum as in amiTermsSource), NUL-terminated into buf as amiTermsSource
 * does.  With compile nonzero it is also compiled for gfx950 with hipRTC (into
 * the disk cache; no device is needed): AMI_E_HIP with the compiler's log
 * when that fails.  AMI_E_UNSUPPORTED when an item is outside the
 * specialized form.
 */
AmiStatus amiBatchSource(AmiTerms *const *terms, int32_t n, const int64_t *n_f, int32_t momentum, int32_t compile,
                         char *buf, int64_t cap, int64_t *len);

/*
 * Kernel timer (measurement): after amiKernelTimerStart(capacity), every
 * evaluate and adjoint call on this thread records a pair of HIP events on its
 * stream around its main kernel (the first `capacity` calls; the row-sum and
 * gradient reduction kernels stay outside).  amiKernelTimerStop waits for the
 * recorded events, writes up to `cap` durations in milliseconds to ms (host)
 * in call order, the number recorded to *count, and releases the events.
 */
AmiStatus amiKernelTimerStart(int32_t capacity);
AmiStatus amiKernelTimerStop(float *ms, int32_t cap, int32_t *count);

/*
 * FP64 fused multiply-add throughput of the current device (measurement, not
 * part of the evaluation): a kernel of eight independent FMA chains per lane
 * for `iters` steps (1..2^24) on 8 blocks of 256 lanes per compute unit,
 * launched twice on `hip_stream`; the second launch is timed with HIP events
 * and *tflops (host) receives 2 * 8 * iters * lanes / seconds / 1e12.  Blocks
 * until done; allocates and frees a small sink buffer.  AMI_E_ARG for a bad
 * iters or NULL tflops, AMI_E_HIP on a HIP error.
 */
AmiStatus amiMeasureFp64Peak(int64_t iters, double *tflops, void *hip_stream);

/* Name of the kernel variant launched by the last evaluate call on this thread. */
const char *amiLastVariant(void);

/*
 * Persistent mixed-diagram batch (one HIP graph launch over many diagrams).
 *
 * Each item is one diagram with its own samples, frequency rows and outputs,
 * exactly as one amiEvaluateHubbard call (k != NULL) or amiEvaluate call
 * (energies != NULL); all items of a batch use the same one of the two paths.
 * Pointers are device pointers on the current device and are baked into the
 * batch at creation: the batch evaluates whatever those buffers hold when it
 * runs.  Every item needs the packed form of its solution (see
 * amiEvaluateAdjoint).
 */
typedef struct AmiBatch AmiBatch;

typedef struct {
    AmiTerms *terms;
    const double *energies;      /* energy path: as amiEvaluate, or NULL       */
    int64_t stride_s, stride_i;
    const double *k;             /* momentum path: as amiEvaluateHubbard, or NULL */
    int64_t stride_k;
    double q[8];                 /* external momenta (2 per external slot)     */
    double t, mu;
    int64_t n_e;                 /* samples (>= 1)                              */
    const double *ext_freqs;     /* complex128 [n_f][n_ext]                     */
    int64_t n_f;
    double beta, e_reg;
    double *out;                 /* complex128 [n_f][n_e] or NULL               */
    double *out_sum;             /* complex128 [n_f] or NULL (not both NULL)    */
} AmiBatchItem;

/* Tuning of a batch (chosen by the autotuner of the Python package):
 *   block        lanes per work-item tile: 64, 128, 256, or 0 for the choice
 *                the packed amiEvaluate makes for the largest item of each class
 *   waves_per_cu resident waves per compute unit of the persistent grid, 1..32
 *   tile_factor  each work item costs about tile_factor times the most
 *                expensive single tile of the batch, 1..1024
 *   kernels      0: every item whose specialized forward an AUTO evaluate call
 *                would run (one or two passes) runs it, the others the packed
 *                persistent kernels; 1: every item on the packed kernels
 *                (block, waves_per_cu and tile_factor tune those only);
 *                2: every item's specialized tile functions inside persistent
 *                kernels (every item needs a specialized forward; block is
 *                ignored, 256 lanes; waves_per_cu caps the resident waves and
 *                tile_factor sizes the work items) */
typedef struct {
    int32_t block;
    int32_t waves_per_cu;
    int32_t tile_factor;
    int32_t kernels;
} AmiBatchTuning;

/*
 * amiBatchCreate -- with tuning.kernels = 0, compile and load the specialized
 * forward of every item that has one (as AUTO would choose it); run those
 * items once, then record their launches from up to four streams (largest
 * first onto the least loaded stream) into a child graph.  Split the other
 * items into LDS classes (equal block size and blocks per CU of their own
 * packed launch, at most 16 classes), build each class's work list (a
 * diagram's sample tiles grouped into items of similar cost, queued from most
 * to least expensive), upload them with the item descriptors, allocate the
 * row-sum workspace, and instantiate the graph (the child graph beside
 * counter reset -> one persistent kernel per class -> fixed-order row sums).
 * All allocation and compilation happens here.  tuning may be NULL (defaults
 * {0, 8, 1, 0}).  An item on its specialized kernels gets out and out_sum
 * equal to an AUTO evaluate call's bit for bit; an item on the packed kernels
 * gets out equal to the packed per-diagram call's (AMI_VARIANT_PACKED) bit for
 * bit, and out_sum too when the class's block size matches that call's.
 * With tuning.kernels = 2: generate, compile (side by side, into the disk
 * cache) and load one module per group of items -- per pass (the one-pass
 * tiles with the two-pass items' first pass, then their frequency pass), the
 * items grouped by the occupancy of their own kernel of that pass -- holding
 * every item's generated tile functions and a persistent kernel that pulls
 * (item, tile range, range of frequency rows) work items from its own
 * counters; the graph runs counter reset -> the first-pass kernels side by
 * side -> the frequency-pass kernels -> fixed-order row sums; out and out_sum
 * equal an AUTO evaluate call's bit for bit.
 */
AmiStatus amiBatchCreate(const AmiBatchItem *items, int32_t n_items, const AmiBatchTuning *tuning,
                         AmiBatch **out);

/* Launch the batch graph on hip_stream (asynchronous; allocates nothing). */
AmiStatus amiBatchRun(AmiBatch *batch, void *hip_stream);

/* info[0..9]: items, work items, grid blocks (summed over the LDS classes),
 * block lanes (of the class with the most work items), LDS bytes per block
 * (largest class), row-sum columns, momentum path (1) or energy path (0),
 * LDS classes (persistent kernels in the graph), items on their specialized
 * kernels, streams their launches were recorded from. */
AmiStatus amiBatchInfo(const AmiBatch *batch, int64_t info[10]);

/* Release a batch (its device workspace and graph). */
void amiBatchFree(AmiBatch *batch);

/* Message of the last failed call on this thread ("" if none). */
const char *amiLastError(void);

/* Library version string. */
const char *amiVersion(void);

#ifdef __cplusplus
}
#endif

#endif /* AMIGPU_H */

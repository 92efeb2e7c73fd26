/*
 * jk_laplace.h -- Laplace pseudo-density driver of the J/K engine (jk.h).
 *
 * The paper, Sec. 2.2 ("The AO-direct Laplace representation", Eq.
 * (laplace)): an orbital-energy denominator x > 0 is the Laplace integral
 * 1/x = int_0^inf exp(-t x) dt, discretized by a short exponential sum
 *
 *     1/x  ~  sum_{k < npts} w_k exp(-alpha_k x),        npts ~ 8-10.
 *
 * Since x is a signed sum of orbital energies (x = e_a - e_i, or
 * e_a + e_b - e_i - e_j, plus a constant shift for a shifted denominator),
 * exp(-alpha_k x) factorizes over the orbital indices, and every
 * denominator-weighted density becomes npts ordinary densities assembled from
 * energy-scaled coefficients C_mp exp(+-alpha_k e_p) (the paper's factor with
 * the exponent split between the two sides of a symmetric pseudo-density is
 * the same call with half the scale).  Each one is an ordinary J/K build.
 *
 * The quadrature is the minimax rule for the RELATIVE error: with
 * y = x / x_min in [1, R], R = x_max / x_min, (w, alpha) minimize
 * max_y |1 - y sum_k w_k exp(-alpha_k y)|.  The paper prints no table and
 * fixes no norm; see jk_laplace_quadrature.
 *
 * Conventions are those of jk.h (device pointers to dense row-major FP64
 * arrays, stream as void*, status codes, nothing written on error).
 */
#ifndef JK_GFX950_LAPLACE_H
#define JK_GFX950_LAPLACE_H

#include "jk.h"

#ifdef __cplusplus
extern "C" {
#endif

enum { JK_LAPLACE_MAX_POINTS = 20 };

/* Exponential-sum rule for 1/x on [x_min, x_max] (host computation, no GPU
 * work; 0.1..5 s, results cached per (npts, x_max/x_min)).
 *   npts          1 .. JK_LAPLACE_MAX_POINTS
 *   x_min, x_max  0 < x_min <= x_max, x_max / x_min <= 1e9; a ratio below 2
 *                 is widened to 2 (a rule for a wider range is valid on the
 *                 narrower one)
 *   w, alpha      HOST arrays of npts doubles, written on success: weights
 *                 and exponents (all > 0), alpha ascending
 *   max_rel_err   HOST pointer or NULL: max over [x_min, x_max] of
 *                 |1 - x sum_k w_k exp(-alpha_k x)|, measured on the returned
 *                 rule (a dense logarithmic scan refined at every local
 *                 extremum), not a nominal value
 *   is_minimax    HOST pointer or NULL: 1 if the relative error
 *                 equioscillates at 2 npts + 1 points with level ripples (the
 *                 best rule of npts terms), else 0 (the best rule the fit
 *                 found; this happens when the range is narrow for npts
 *                 terms and the error is already below about 1e-6)
 * Method: trapezoid start in the substitution t = e^s, least p-th powers of
 * the relative error on a logarithmic grid for p = 2 .. 64
 * (Levenberg-Marquardt), then Remez exchange: Newton's method on the
 * 2 npts + 1 equioscillation equations, the reference moved to the extrema
 * of the new error curve until they are level.  Returns JK_EINVAL on bad
 * arguments, JK_OK otherwise. */
jk_status jk_laplace_quadrature(int32_t npts, double x_min, double x_max, double *w,
                                double *alpha, double *max_rel_err, int32_t *is_minimax);

/* Energy-scaled factors (Sec. 2.2): for k < npts, m < nvec,
 *     out[k][m][mu][i] = coef_k * sum_a C[mu][a] exp(scale alpha_k e[a]) X_m[i][a]
 * or, with X == NULL (then rank must equal norb),
 *     out[k][m][mu][i] = coef_k * C[mu][i] exp(scale alpha_k e[i])
 * (the same for every m).
 *   C      DEVICE [nao][norb]       orbital coefficients
 *   e      DEVICE [norb]            orbital energies
 *   X      DEVICE [nvec][rank][norb] or NULL
 *   alpha, coef  HOST arrays of npts doubles (copied into the launch)
 *   out    DEVICE [npts][nvec][nao][rank], overwritten
 * Sizes: 1 <= nao <= 16384, 1 <= norb, rank <= 16384, 1 <= nvec, 1 <= npts
 * <= JK_LAPLACE_MAX_POINTS, npts * nvec * nao * rank < 2^40.  The exponential
 * is evaluated in FP64 per element; a factor that overflows is the caller's
 * range problem (the product of the two sides of a pseudo-density is always
 * exp(-alpha_k x) <= 1 for x > 0).  The X contraction runs on the FP64
 * matrix cores; the sum over a is in a fixed order. */
jk_status jk_laplace_factors(int64_t nao, int64_t norb, int64_t rank, int64_t nvec, int32_t npts,
                             const double *C, const double *e, const double *X,
                             const double *alpha, const double *coef, double scale, double *out,
                             void *stream);

typedef struct {
    int64_t nao;       /* basis size                                         */
    int64_t naux;      /* Cholesky vectors                                   */
    int64_t nocc;      /* columns of Cocc (index i), 1 <= nocc <= nao         */
    int64_t nvir;      /* columns of Cvir (index a), >= 1                    */
    int64_t nvec;      /* amplitude matrices X_m, >= 1                       */
    int32_t npts;      /* quadrature points, 1 .. JK_LAPLACE_MAX_POINTS       */
    int32_t precision; /* jk_precision of the J/K builds                     */
    int32_t flags;     /* JK_WANT_J | JK_WANT_K (0 means both)               */
    int32_t nslice;    /* as in jk_problem                                   */
} jk_laplace_problem;

/* Workspace bytes for jk_laplace_build (0 if *p is invalid). */
size_t jk_laplace_workspace_bytes(const jk_laplace_problem *p);

/* Transition pseudo-densities (Sec. 2.2 with the non-symmetric kernel of
 * Sec. 2.3): for k < npts, m < nvec, with c_k = w_k exp(-alpha_k shift),
 *     D_km = c_k Cocc diag(exp(+alpha_k e_occ)) X_m diag(exp(-alpha_k e_vir)) Cvir^T
 *          = CL_km CR_km^T,  CL_km = c_k Cocc exp(+alpha_k e_occ)   [nao][nocc]
 *                            CR_km = Cvir exp(-alpha_k e_vir) X_m^T [nao][nocc]
 * and J_km = J[D_km], K_km = K[D_km] as in jk_build (ndens = npts * nvec,
 * rank = nocc, density index k * nvec + m).  With a rule fitted on a range
 * that holds every e_a - e_i + shift, the sum over k of D_km approximates
 * Cocc (X_m / (e_a - e_i + shift)) Cvir^T, each element within the rule's
 * relative error; with a rule for the range of e_a + e_b - e_i - e_j +
 * shift, projecting J_km, K_km on the orbitals and scaling by
 * exp(alpha_k (e_i - e_a)) gives the doubles-denominator contractions of
 * Eq. (laplace) (sum over k of the scaled projections).
 *   B            DEVICE [naux][nao][nao] (symmetric slabs, as in jk.h)
 *   Cocc         DEVICE [nao][nocc],   e_occ DEVICE [nocc]
 *   Cvir         DEVICE [nao][nvir],   e_vir DEVICE [nvir]
 *   X            DEVICE [nvec][nocc][nvir]
 *   w, alpha     HOST arrays of npts doubles (e.g. jk_laplace_quadrature)
 *   J, K         DEVICE [npts][nvec][nao][nao], as selected by flags
 * The factors live in the workspace; nothing else is allocated. */
jk_status jk_laplace_build(const jk_laplace_problem *p, const double *B, const double *Cocc,
                           const double *e_occ, const double *Cvir, const double *e_vir,
                           const double *X, const double *w, const double *alpha, double shift,
                           double *J, double *K, void *ws, size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif

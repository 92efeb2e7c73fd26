/*
 * jk.h -- C ABI of the MI355X (gfx950) Cholesky-decomposed Coulomb/exchange
 * engine for non-symmetric densities.
 *
 * The operation (the paper, Sec. 2.3 "The non-symmetric AO-Laplace J/K
 * kernel", Eq. (4), in the Cholesky-decomposed representation
 * (mn|ls) = sum_Q B^Q_mn B^Q_ls and the half-transform form K = B_V^T B_U
 * stated in the same section): for densities D_k = C_Lk C_Rk^T, k < ndens,
 *
 *     gamma_kQ = <B^Q, D_k>               (Frobenius pairing)
 *     J_k      = sum_Q gamma_kQ B^Q
 *     K_k      = sum_Q B^Q D_k B^Q  = sum_Q (B^Q C_Lk) (B^Q C_Rk)^T
 *
 * and the reverse-mode derivative of L = sum_k <Jbar_k, J_k> + <Kbar_k, K_k>
 * (Sec. 2.1, Eq. (1): the adjoint of J and K is J and K of the cotangent).
 *
 * Conventions shared by every entry point
 *   - All array arguments are DEVICE pointers to caller-owned FP64 memory,
 *     row-major and densely packed:
 *        B          [naux][nao][nao]     every slab B^Q symmetric (precondition,
 *                                        not checked; the kernels read B^Q as
 *                                        its own transpose)
 *        CL, CR     [ndens][nao][rank]
 *        J, K       [ndens][nao][nao]    outputs, overwritten (never accumulated)
 *        Jbar, Kbar [ndens][nao][nao]    cotangents W_k, V_k (need not be symmetric)
 *        dB         [naux][nao][nao]     dL/dB, the literal-formula gradient
 *                                        (see jk_vjp)
 *        dCL, dCR   [ndens][nao][rank]
 *   - ws/ws_bytes: a caller-provided DEVICE workspace of at least the size the
 *     matching *_workspace_bytes query returns.  The library allocates no
 *     device memory in these calls.  ws must be 256-byte aligned.
 *   - stream: a hipStream_t passed as void* (NULL = the default stream).  All
 *     work is enqueued on it; calls return without synchronising the host.
 *   - Errors: arguments are validated before anything is enqueued; on any
 *     error status nothing is written.  A failed launch returns JK_EHIP;
 *     a failed host allocation (plans, schedules, tables) returns JK_ENOMEM.
 *     Faults of already-enqueued kernels surface at the caller's next
 *     synchronisation.  No C++ exception crosses this interface.
 *   - Buffers of one call must not overlap, except that inputs may alias
 *     inputs.  Concurrent calls on different streams need separate workspaces.
 *   - Results are deterministic: the same inputs and problem give bit-identical
 *     outputs (no floating-point atomics; every sum has a fixed order).
 */
#ifndef JK_GFX950_H
#define JK_GFX950_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    JK_OK = 0,
    JK_EINVAL = 1,        /* bad size, null required pointer, misaligned ws  */
    JK_EWORKSPACE = 2,    /* ws_bytes below the required size                */
    JK_EUNSUPPORTED = 3,  /* valid but not implemented combination           */
    JK_EHIP = 4,          /* a HIP launch or runtime call failed             */
    JK_ENOMEM = 5         /* host-side bookkeeping could not be allocated     */
} jk_status;

typedef enum {
    JK_FP64 = 0,   /* every product and sum in FP64                          */
    JK_MIXED = 1   /* half-transforms and K products on the INT8 matrix
                      cores as exact fixed-point slice products: each row
                      gets one power-of-two scale 2^e (max|row| <=
                      2^e 127/128) and each value the 31-bit integer
                      rint(a 2^(31-e)), written as 4 balanced base-256
                      digits; the 13 digit pairs with i + j <= 6 are
                      multiplied with int32 accumulation.  FP64 for gamma,
                      J, the recombination of the digit levels (power-of-
                      two weights), every cross-chunk sum and the final
                      accumulation.  Normwise error of K about 1e-9 on
                      smoothly scaled inputs; rows whose inner-index
                      magnitudes span many orders of magnitude lose the
                      small entries (fixed point).
                      Exactness of the int32 sums: |digit| <= 128, and a
                      level adds at most 4 digit pairs per inner index, so
                      a sum over n indices stays below 2^31 for
                      n <= 32767; the planner splits every contraction to
                      at most that depth (jk_plan_describe in jk_tune.h
                      reports it).                                           */
} jk_precision;

/* JK_B_PACKED: every B slab (and B_lr slab of jk_fock) is stored as its upper
 * triangle, row by row: element (m, n), m <= n, of slab Q at
 * Q * nao (nao + 1) / 2 + m nao - m (m - 1) / 2 + (n - m), so B takes
 * naux nao (nao + 1) / 2 doubles, half the full square.  gamma and J stream
 * the packed positions (half the bytes); the half-transforms read each
 * element (m, n) at its packed place.  Accepted by jk_build, jk_fock and
 * jk_laplace_build and jk_build_batched (FP64 and JK_MIXED; mixed needs
 * nao <= 2048) and by jk_vjp (FP64; dB then comes back packed too). */
enum { JK_WANT_J = 1, JK_WANT_K = 2, JK_B_PACKED = 4 };

typedef struct {
    int64_t nao;       /* basis size, >= 1                                   */
    int64_t naux;      /* number of Cholesky vectors Q, >= 1                 */
    int64_t ndens;     /* number of densities k, >= 1                        */
    int64_t rank;      /* columns of each CL_k / CR_k, 1 <= rank <= nao      */
    int32_t precision; /* jk_precision                                       */
    int32_t flags;     /* JK_WANT_J | JK_WANT_K (neither means both),
                          optionally | JK_B_PACKED                           */
    int32_t nslice;    /* JK_MIXED only: digits per operand; 0 or 4 (the
                          one implemented value; 1..3 and 5 give
                          JK_EUNSUPPORTED)                                   */
    int32_t reserved;  /* must be 0                                          */
} jk_problem;

/* Workspace bytes needed by jk_build and jk_vjp for problem *p (one size
 * serves both).  Returns 0 if *p is invalid. */
size_t jk_workspace_bytes(const jk_problem *p);

/* Forward build (Sec. 2.3, Eq. (4)): J_k and K_k for every density k.
 * Writes J if flags has JK_WANT_J (J may be NULL otherwise) and K if flags
 * has JK_WANT_K (K may be NULL otherwise).
 * Symmetric densities: when CL and CR are the same pointer, every D_k =
 * C_k C_k^T is symmetric (the C_L = C_R case of Sec. 2.3); only X = B^Q C is
 * formed and K_k = sum_Q X X^T is computed on its upper triangle and
 * mirrored, so K is exactly symmetric.  Equal contents behind two different
 * pointers take the general path. */
jk_status jk_build(const jk_problem *p, const double *B, const double *CL,
                   const double *CR, double *J, double *K, void *ws,
                   size_t ws_bytes, void *stream);

/* Digit planes of B for JK_MIXED, made once and reused by every build over
 * the same B.  The consumers of the paper rebuild J and K many times on one
 * set of Cholesky vectors (Sec. 2.1: the Z-vector iterations; Sec. 2.2: one
 * build per Laplace point), so slicing B (reading its FP64 values and
 * writing the integer planes) need not be repeated.
 *   jk_slices_bytes   size of the buffer for problem *p (0 if *p is invalid
 *                     or not JK_MIXED).  It depends on nao and naux only:
 *                     about 4 bytes per element of B plus padding to 64
 *                     rows and 32 columns per slab.
 *   jk_slice_b        writes the planes of B (full or packed slabs, as
 *                     p->flags says) into `slices` (DEVICE, 256-byte aligned,
 *                     caller-owned), on the stream.
 *   jk_build_sliced   jk_build with JK_MIXED that reads the half-transforms'
 *                     B operand from `slices` instead of slicing B again; B
 *                     itself is still read for gamma and J (FP64).  Same
 *                     workspace as jk_build (jk_workspace_bytes).  The
 *                     results are bit-identical to jk_build's.  `slices`
 *                     must have been made by jk_slice_b from this B with the
 *                     same nao, naux and layout flag (not checked); a B that
 *                     changes needs new slices.
 * Errors as jk_build; JK_EINVAL for a precision other than JK_MIXED. */
size_t jk_slices_bytes(const jk_problem *p);
jk_status jk_slice_b(const jk_problem *p, const double *B, void *slices, size_t slices_bytes,
                     void *stream);
jk_status jk_build_sliced(const jk_problem *p, const double *B, const void *slices,
                          size_t slices_bytes, const double *CL, const double *CR, double *J,
                          double *K, void *ws, size_t ws_bytes, void *stream);

/* jk_build without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same operation, arguments, outputs and symmetric-density
 * rule as jk_build; the caller still passes B, CL, CR, J and K.  Every kernel
 * buffer lives in a 256 MiB array of device memory inside the library, one
 * per GPU, held until the process ends; the call allocates nothing.
 *   - JK_FP64 only (full or packed slabs); JK_MIXED gives JK_EUNSUPPORTED.
 *   - Problems whose smallest plan needs more than 256 MiB return
 *     JK_EWORKSPACE before anything is enqueued (for example nao = 1000 with
 *     16 densities of rank 80 fits, in chunks of a few slabs; nao = 2000 with
 *     16 densities, whose densities alone take 512 MB, does not).
 *   - The plan is the recorded tile (jk_tune.h) with the largest chunk budget
 *     up to 256 MiB that fits, so K agrees with jk_build to rounding.
 *   - All calls on one GPU share that GPU's array: calls that overlap in time
 *     on one GPU (different streams, or threads) race and give wrong
 *     results; serialise them.  No buffer needs to start at zero. */
jk_status jk_build_noalloc(const jk_problem *p, const double *B, const double *CL,
                           const double *CR, double *J, double *K, void *stream);

/* Workspace bytes needed by jk_fock for problem *p (0 if invalid). */
size_t jk_fock_workspace_bytes(const jk_problem *p, int64_t naux_lr);

/* Fock-type combination in one call (Sec. 2.1, Eq. (selfadjoint): J, K and
 * the long-range exchange K_LR are nodes of one self-adjoint family; Sec.
 * 2.6 and Sec. 4.1: the combination 2J - a_x K of the SCF response and of
 * the derivative Fock build; Sec. 2.5: range-separated exchange through
 * K_LR):
 *     F_k = c_j J[D_k] + c_k K[D_k] + c_lr K_lr[D_k],   D_k = CL_k CR_k^T,
 *     K_lr[D] = sum_P B_lr^P D B_lr^P  with a second Cholesky factor set
 *               B_lr [naux_lr][nao][nao] (symmetric slabs), e.g. that of the
 *               long-range Coulomb operator.
 * Both exchange streams accumulate into one set of partial sums (every
 * chunk's contribution scaled by its coefficient), and J is added by the
 * Coulomb pass at the end: F is the only output array written.
 *   coef   HOST array {c_j, c_k, c_lr}; a zero coefficient skips its term
 *          (all zero: F = 0)
 *   B_lr   DEVICE pointer or NULL; NULL requires naux_lr == 0 and c_lr == 0
 *   F      DEVICE [ndens][nao][nao], overwritten
 * p->flags must request both J and K (0, or JK_WANT_J | JK_WANT_K), with or
 * without JK_B_PACKED.  FP64 and JK_MIXED (the
 * exchange products of both streams in INT8 slices, J in FP64).  CL == CR
 * takes the symmetric path as in jk_build.  Summation order differs from
 * adding separate jk_build results, so F agrees with them to rounding, not
 * bit for bit. */
jk_status jk_fock(const jk_problem *p, const double *B, const double *B_lr, int64_t naux_lr,
                  const double *CL, const double *CR, const double *coef, double *F, void *ws,
                  size_t ws_bytes, void *stream);

/* Workspace bytes needed by jk_build_batched for the nprob problems p[0..]. */
size_t jk_batched_workspace_bytes(int32_t nprob, const jk_problem *p);

/* Many independent problems (geometries of uneven size, each with its own
 * nao, naux, ndens and rank) in one call.  p, B, CL, CR, J, K are HOST arrays
 * of length nprob; B[g], CL[g], ... are DEVICE pointers with the layouts
 * above.  Every problem must share one precision and one flags value.  Each
 * member's outputs agree with a jk_build call of that member alone to
 * rounding, and are bit-identical to it when that build's plan (jk_tune.h)
 * has a chunk budget of at most 1 GiB (JK_FP64) or 256 MiB (JK_MIXED): each
 * member's Q-chunks are capped at that budget, and K sums its chunks in
 * order.  Every member owns its chunk buffers, so the workspace grows with
 * the members (53 GiB for 64 FP64 geometries of nao 100..500, naux = 4 nao,
 * 6 densities of rank nao/10).  With a non-default stream the
 * launch sequence is captured once per shape signature, workspace and device
 * and replayed (at most 32 such graphs are kept; the oldest is destroyed,
 * after a device synchronisation, when a new one is made).  The member
 * table is copied from a pinned host buffer that the library owns. */
jk_status jk_build_batched(int32_t nprob, const jk_problem *p,
                           const double *const *B, const double *const *CL,
                           const double *const *CR, double *const *J,
                           double *const *K, void *ws, size_t ws_bytes,
                           void *stream);

/* Reverse-mode derivative (Sec. 2.1, Eq. (1)) of
 *     L = sum_k <Jbar_k, J_k> + <Kbar_k, K_k>
 * with W_k = Jbar_k, V_k = Kbar_k (either may be NULL = zero cotangent):
 *     omega_kQ = <W_k, B^Q>,  X^Q_k = B^Q CL_k,  Y^Q_k = B^Q CR_k
 *     dCL_k = sum_Q B^Q (V_k Y^Q_k)   + omega_kQ Y^Q_k
 *     dCR_k = sum_Q B^Q (V_k^T X^Q_k) + omega_kQ X^Q_k
 *     dB^Q  = sum_k gamma_kQ W_k + omega_kQ D_k + V_k B^Q D_k^T + D_k^T B^Q V_k
 * dB is the gradient of the literal formulas for a general B evaluated at the
 * given symmetric B (its symmetric part is convention-free).  The
 * half-transforms are recomputed, not stored.  dB may be NULL (not computed);
 * dCL and dCR are both NULL (not computed) or both non-NULL (else
 * JK_EINVAL).  Only JK_FP64 is supported, and one slab's block of factor
 * columns must stay below 4 GiB: 16 nao ndens rank < 2^32 bytes (else
 * JK_EUNSUPPORTED).
 * Packed B (JK_B_PACKED): dB has B's packed layout and holds the gradient
 * with respect to the packed elements, dB[m][n] + dB[n][m] at (m, n), m < n,
 * and dB[m][m] on the diagonal.  The projections stream the packed slabs;
 * each Q-chunk is unpacked into a workspace buffer of full squares that the
 * half-transforms and the products B^Q [P' | R'] read (the workspace grows by
 * chunk slabs x 8 nao^2 bytes).
 * Symmetric densities: when CL and CR are the same pointer (the C_L = C_R
 * case of Sec. 2.3), Y^Q_k = X^Q_k, so only X is recomputed and both products
 * V_k Y and V_k^T X read it.  dCL and dCR are still the two separate
 * gradients (their sum is the gradient with respect to the shared factor),
 * bit-identical to those of the general path given equal contents behind two
 * pointers. */
jk_status jk_vjp(const jk_problem *p, const double *B, const double *CL,
                 const double *CR, const double *Jbar, const double *Kbar,
                 double *dB, double *dCL, double *dCR, void *ws,
                 size_t ws_bytes, void *stream);

/* Static, NUL-terminated description of a status code. */
const char *jk_status_str(jk_status s);

#ifdef __cplusplus
}
#endif
#endif /* JK_GFX950_H */

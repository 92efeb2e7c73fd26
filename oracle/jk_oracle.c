/*
 * jk_oracle.c -- plain, slow, FP64 CPU oracle for the Cholesky-decomposed
 * Coulomb/exchange (J/K) build with non-symmetric densities, its reverse-mode
 * vector-Jacobian product and its forward-mode derivative.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent reference that the
 * GPU library is checked against.  Only the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.  It shares no code,
 * header, table or constant with the HIP library and includes nothing of it.
 *
 * What is computed (the paper: Sec. 2.3 "The non-symmetric AO-Laplace J/K
 * kernel", Eq. (4); the Cholesky-decomposed representation and the
 * half-transform form K = B_V^T B_U stated in the same section):
 *
 *   (mn|ls)     = sum_Q B^Q_mn B^Q_ls                    Cholesky factorisation
 *   D_k         = C_Lk C_Rk^T                            factored density
 *   gamma_kQ    = sum_ls B^Q_ls D_k,ls                   Coulomb vector
 *   J_k,mn      = sum_Q gamma_kQ B^Q_mn = sum_ls (mn|ls) D_k,ls
 *   K_k,mn      = sum_Q sum_ls B^Q_ml D_k,ls B^Q_sn = sum_ls (ml|sn) D_k,ls
 *
 * Derivatives (Sec. 2.1, Eq. (1): the adjoint of J and K is J and K applied
 * to the cotangent).  For the scalar L = sum_k <W_k,J_k> + <V_k,K_k> with the
 * Frobenius pairing <A,B> = tr(A^T B), differentiating the formulas above for
 * a general (not necessarily symmetric) B gives
 *
 *   omega_kQ    = <W_k, B^Q>
 *   dL/dD_k     = sum_Q omega_kQ B^Q + B^Q^T V_k B^Q^T
 *   dL/dC_Lk    = (dL/dD_k) C_Rk
 *   dL/dC_Rk    = (dL/dD_k)^T C_Lk
 *   dL/dB^Q     = sum_k gamma_kQ W_k + omega_kQ D_k
 *                       + V_k B^Q^T D_k^T + D_k^T B^Q^T V_k
 *
 * Layouts (row-major, host memory, caller-owned):
 *   B   [naux][nao][nao]        CL, CR [nd][nao][r]
 *   D   [nd][nao][nao]          J, K, W, V, dB-per-density [nd][nao][nao]
 *   gamma, omega [nd][naux]     eri [nao][nao][nao][nao]
 *
 * Tiers: T0 brute force through the explicit 4-index tensor; T1 the plain
 * definition with explicit D and literal matrix products; T2 the factored
 * (half-transform) rearrangement; T3 single entries computed one by one.
 *
 * Loops are plain and parallelised with OpenMP over independent outputs only,
 * so every output element is summed by one thread in a fixed order.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef int64_t i64;

#define B_AT(B, nao, q, m, n) ((B)[((i64)(q) * (nao) + (m)) * (nao) + (n)])

/* ------------------------------------------------------------------ T0 */

/* (mn|ls) = sum_Q B^Q_mn B^Q_ls : the 4-index tensor the Cholesky factor
 * represents (Sec. 2.3). */
void jko_eri4(i64 nao, i64 naux, const double *B, double *eri)
{
    i64 n2 = nao * nao;
#pragma omp parallel for schedule(static)
    for (i64 mn = 0; mn < n2; mn++) {
        for (i64 ls = 0; ls < n2; ls++) {
            double s = 0.0;
            for (i64 q = 0; q < naux; q++)
                s += B[q * n2 + mn] * B[q * n2 + ls];
            eri[mn * n2 + ls] = s;
        }
    }
}

/* J_mn = sum_ls (mn|ls) D_ls ; K_mn = sum_ls (ml|sn) D_ls  (Eq. (4) with one
 * weight density contracted, the other index pair left open). */
void jko_jk_from_eri(i64 nao, const double *eri, const double *D,
                     double *J, double *K)
{
    i64 n2 = nao * nao;
#pragma omp parallel for schedule(static)
    for (i64 m = 0; m < nao; m++) {
        for (i64 n = 0; n < nao; n++) {
            double sj = 0.0, sk = 0.0;
            for (i64 l = 0; l < nao; l++) {
                for (i64 s = 0; s < nao; s++) {
                    double d = D[l * nao + s];
                    sj += eri[(m * nao + n) * n2 + l * nao + s] * d;
                    sk += eri[(m * nao + l) * n2 + s * nao + n] * d;
                }
            }
            J[m * nao + n] = sj;
            K[m * nao + n] = sk;
        }
    }
}

/* ------------------------------------------------------------------ T1 */

/* D_k = C_Lk C_Rk^T for every density k. */
void jko_density(i64 nd, i64 nao, i64 r, const double *CL, const double *CR,
                 double *D)
{
#pragma omp parallel for collapse(2) schedule(static)
    for (i64 k = 0; k < nd; k++) {
        for (i64 m = 0; m < nao; m++) {
            const double *cl = CL + (k * nao + m) * r;
            for (i64 n = 0; n < nao; n++) {
                const double *cr = CR + (k * nao + n) * r;
                double s = 0.0;
                for (i64 i = 0; i < r; i++)
                    s += cl[i] * cr[i];
                D[(k * nao + m) * nao + n] = s;
            }
        }
    }
}

/* g_kQ = <A_k, B^Q> = sum_ls B^Q_ls A_k,ls.  With A = D this is the Coulomb
 * vector gamma; with A = W it is the cotangent projection omega. */
void jko_project(i64 nd, i64 nao, i64 naux, const double *B, const double *A,
                 double *g)
{
    i64 n2 = nao * nao;
#pragma omp parallel for collapse(2) schedule(static)
    for (i64 k = 0; k < nd; k++) {
        for (i64 q = 0; q < naux; q++) {
            double s = 0.0;
            for (i64 ls = 0; ls < n2; ls++)
                s += B[q * n2 + ls] * A[k * n2 + ls];
            g[k * naux + q] = s;
        }
    }
}

/* J_k = sum_Q g_kQ B^Q. */
void jko_coulomb(i64 nd, i64 nao, i64 naux, const double *B, const double *g,
                 double *J)
{
    i64 n2 = nao * nao;
#pragma omp parallel for collapse(2) schedule(static)
    for (i64 k = 0; k < nd; k++) {
        for (i64 mn = 0; mn < n2; mn++) {
            double s = 0.0;
            for (i64 q = 0; q < naux; q++)
                s += g[k * naux + q] * B[q * n2 + mn];
            J[k * n2 + mn] = s;
        }
    }
}

/* K_k = sum_Q B^Q D_k B^Q as literal matrix products (the index form of the
 * exchange operator, Sec. 2.3).  Per (k, Q): T = D_k B^Q, then B^Q T.
 * Works for a general (non-symmetric) B. */
void jko_exchange(i64 nd, i64 nao, i64 naux, const double *B, const double *D,
                  double *K)
{
    i64 n2 = nao * nao;
    double *T = (double *)malloc(sizeof(double) * n2);
    for (i64 k = 0; k < nd; k++) {
        const double *Dk = D + k * n2;
        double *acc = K + k * n2;
        for (i64 e = 0; e < n2; e++)
            acc[e] = 0.0;
        for (i64 q = 0; q < naux; q++) {
            const double *Bq = B + q * n2;
            /* T_ln = sum_t D_lt B_tn */
#pragma omp parallel for schedule(static)
            for (i64 l = 0; l < nao; l++)
                for (i64 n = 0; n < nao; n++) {
                    double s = 0.0;
                    for (i64 t = 0; t < nao; t++)
                        s += Dk[l * nao + t] * Bq[t * nao + n];
                    T[l * nao + n] = s;
                }
            /* acc_mn += sum_l B_ml T_ln */
#pragma omp parallel for schedule(static)
            for (i64 m = 0; m < nao; m++)
                for (i64 n = 0; n < nao; n++) {
                    double s = 0.0;
                    for (i64 l = 0; l < nao; l++)
                        s += Bq[m * nao + l] * T[l * nao + n];
                    acc[m * nao + n] += s;
                }
        }
    }
    free(T);
}

/* ------------------------------------------------------------------ T2 */

/* Factored build (the half-transform form of Sec. 2.3, K = B_V^T B_U): with
 * symmetric B^Q, for every density k and slab Q
 *   X^Q_k = B^Q C_Lk,  Y^Q_k = B^Q C_Rk,
 *   gamma_kQ = <C_Lk, Y^Q_k>,  K_k += X^Q_k (Y^Q_k)^T,
 * and finally J_k = sum_Q gamma_kQ B^Q.  An exact rearrangement of T1 for
 * symmetric B.  Each half-transform is formed once (6 naux nao^2 R flops, the
 * cost the method itself pays).  Q is summed in increasing order; threads
 * split rows only.  gamma is written if gamma_out is non-NULL. */
void jko_jk_factored(i64 nd, i64 nao, i64 naux, i64 r, const double *B,
                     const double *CL, const double *CR, double *J, double *K,
                     double *gamma_out)
{
    i64 n2 = nao * nao;
    double *gam = (double *)malloc(sizeof(double) * nd * naux);
    double *x = (double *)malloc(sizeof(double) * nao * r);
    double *y = (double *)malloc(sizeof(double) * nao * r);
    for (i64 k = 0; k < nd; k++) {
        const double *cl = CL + k * nao * r, *cr = CR + k * nao * r;
        double *Kk = K + k * n2;
        for (i64 e = 0; e < n2; e++)
            Kk[e] = 0.0;
        for (i64 q = 0; q < naux; q++) {
            const double *Bq = B + q * n2;
#pragma omp parallel for schedule(static)
            for (i64 m = 0; m < nao; m++) {
                double *xm = x + m * r, *ym = y + m * r;
                for (i64 i = 0; i < r; i++) {
                    xm[i] = 0.0;
                    ym[i] = 0.0;
                }
                for (i64 l = 0; l < nao; l++) {
                    double b = Bq[m * nao + l];
                    for (i64 i = 0; i < r; i++) {
                        xm[i] += b * cl[l * r + i];
                        ym[i] += b * cr[l * r + i];
                    }
                }
            }
            double g = 0.0;
            for (i64 m = 0; m < nao; m++)
                for (i64 i = 0; i < r; i++)
                    g += cl[m * r + i] * y[m * r + i];
            gam[k * naux + q] = g;
#pragma omp parallel for schedule(static)
            for (i64 m = 0; m < nao; m++)
                for (i64 n = 0; n < nao; n++) {
                    double s = 0.0;
                    for (i64 i = 0; i < r; i++)
                        s += x[m * r + i] * y[n * r + i];
                    Kk[m * nao + n] += s;
                }
        }
    }
    jko_coulomb(nd, nao, naux, B, gam, J);
    if (gamma_out)
        memcpy(gamma_out, gam, sizeof(double) * nd * naux);
    free(gam);
    free(x);
    free(y);
}

/* ------------------------------------------------------------------ T3 */

/* Single entries, each summed on its own (for inputs too large for the full
 * oracle).  For entry e: density ks[e], row ms[e], column ns[e], Q over
 * [0, naux).  Symmetric B is assumed, as in the factored form:
 *   K_k,mn = sum_Q (B^Q[m,:] C_Lk) . (B^Q[n,:] C_Rk)
 *   J_k,mn = sum_Q gamma_kQ B^Q_mn
 * gamma [nd][naux] is an input (from jko_project with D = C_L C_R^T). */
void jko_jk_entries(i64 nao, i64 naux, i64 r, const double *B,
                    const double *CL, const double *CR, const double *gamma,
                    i64 nent, const i64 *ks, const i64 *ms, const i64 *ns,
                    double *Jout, double *Kout)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (i64 e = 0; e < nent; e++) {
        i64 k = ks[e], m = ms[e], n = ns[e];
        const double *cl = CL + k * nao * r, *cr = CR + k * nao * r;
        double sj = 0.0, sk = 0.0;
        for (i64 q = 0; q < naux; q++) {
            double kq = 0.0;
            for (i64 i = 0; i < r; i++) {
                double sx = 0.0, sy = 0.0;
                for (i64 l = 0; l < nao; l++) {
                    sx += B_AT(B, nao, q, m, l) * cl[l * r + i];
                    sy += B_AT(B, nao, q, n, l) * cr[l * r + i];
                }
                kq += sx * sy;
            }
            sk += kq;
            sj += gamma[k * naux + q] * B_AT(B, nao, q, m, n);
        }
        Jout[e] = sj;
        Kout[e] = sk;
    }
}

/* ----------------------------------------------------------- VJP (Eq. 1) */

/* Reverse-mode derivative of L = sum_k <W_k,J_k> + <V_k,K_k> with respect to
 * B, C_L and C_R, from the literal formulas for a general B (see header).
 * W or V may be NULL (zero cotangent); dB, dCL, dCR may be NULL (skipped). */
void jko_vjp(i64 nd, i64 nao, i64 naux, i64 r, const double *B,
             const double *CL, const double *CR, const double *W,
             const double *V, double *dB, double *dCL, double *dCR)
{
    i64 n2 = nao * nao;
    double *D = (double *)malloc(sizeof(double) * nd * n2);
    double *gam = (double *)malloc(sizeof(double) * nd * naux);
    double *om = (double *)calloc(nd * naux, sizeof(double));
    double *dD = (double *)calloc(nd * n2, sizeof(double));
    jko_density(nd, nao, r, CL, CR, D);
    jko_project(nd, nao, naux, B, D, gam);
    if (W)
        jko_project(nd, nao, naux, B, W, om);

    /* dL/dD_k = sum_Q omega_kQ B^Q + B^Q^T V_k B^Q^T */
    double *T = (double *)malloc(sizeof(double) * n2);
    for (i64 k = 0; k < nd; k++) {
        double *acc = dD + k * n2;
        for (i64 q = 0; q < naux; q++) {
            const double *Bq = B + q * n2;
            double w = om[k * naux + q];
            for (i64 ls = 0; ls < n2; ls++)
                acc[ls] += w * Bq[ls];
            if (!V)
                continue;
            const double *Vk = V + k * n2;
            /* T_ms = sum_n V_mn (B^T)_ns = sum_n V_mn B_sn */
#pragma omp parallel for schedule(static)
            for (i64 m = 0; m < nao; m++)
                for (i64 s = 0; s < nao; s++) {
                    double t = 0.0;
                    for (i64 n = 0; n < nao; n++)
                        t += Vk[m * nao + n] * Bq[s * nao + n];
                    T[m * nao + s] = t;
                }
            /* acc_ls += sum_m (B^T)_lm T_ms = sum_m B_ml T_ms */
#pragma omp parallel for schedule(static)
            for (i64 l = 0; l < nao; l++)
                for (i64 s = 0; s < nao; s++) {
                    double t = 0.0;
                    for (i64 m = 0; m < nao; m++)
                        t += Bq[m * nao + l] * T[m * nao + s];
                    acc[l * nao + s] += t;
                }
        }
    }
    free(T);

    /* dC_Lk = dD_k C_Rk ; dC_Rk = dD_k^T C_Lk */
    if (dCL || dCR) {
#pragma omp parallel for collapse(2) schedule(static)
        for (i64 k = 0; k < nd; k++) {
            for (i64 m = 0; m < nao; m++) {
                for (i64 i = 0; i < r; i++) {
                    double sl = 0.0, sr = 0.0;
                    for (i64 n = 0; n < nao; n++) {
                        sl += dD[(k * nao + m) * nao + n] * CR[(k * nao + n) * r + i];
                        sr += dD[(k * nao + n) * nao + m] * CL[(k * nao + n) * r + i];
                    }
                    if (dCL)
                        dCL[(k * nao + m) * r + i] = sl;
                    if (dCR)
                        dCR[(k * nao + m) * r + i] = sr;
                }
            }
        }
    }

    /* dB^Q = sum_k gamma_kQ W_k + omega_kQ D_k + V_k B^Q^T D_k^T
     *              + D_k^T B^Q^T V_k                                        */
    if (dB) {
#pragma omp parallel for schedule(static)
        for (i64 q = 0; q < naux; q++) {
            const double *Bq = B + q * n2;
            double *out = dB + q * n2;
            double *T = (double *)malloc(sizeof(double) * n2);
            double *U = (double *)malloc(sizeof(double) * n2);
            for (i64 ab = 0; ab < n2; ab++)
                out[ab] = 0.0;
            for (i64 k = 0; k < nd; k++) {
                const double *Dk = D + k * n2;
                double g = gam[k * naux + q], w = om[k * naux + q];
                for (i64 ab = 0; ab < n2; ab++) {
                    double v = w * Dk[ab];
                    if (W)
                        v += g * W[k * n2 + ab];
                    out[ab] += v;
                }
                if (!V)
                    continue;
                const double *Vk = V + k * n2;
                /* T = B^T D^T : T_cb = sum_d B_dc D_bd */
                for (i64 c = 0; c < nao; c++)
                    for (i64 b = 0; b < nao; b++) {
                        double t = 0.0;
                        for (i64 d = 0; d < nao; d++)
                            t += Bq[d * nao + c] * Dk[b * nao + d];
                        T[c * nao + b] = t;
                    }
                /* U = B^T V : U_cb = sum_d B_dc V_db */
                for (i64 c = 0; c < nao; c++)
                    for (i64 b = 0; b < nao; b++) {
                        double t = 0.0;
                        for (i64 d = 0; d < nao; d++)
                            t += Bq[d * nao + c] * Vk[d * nao + b];
                        U[c * nao + b] = t;
                    }
                /* out_ab += sum_c V_ac T_cb + sum_c D_ca U_cb */
                for (i64 a = 0; a < nao; a++)
                    for (i64 b = 0; b < nao; b++) {
                        double t = 0.0;
                        for (i64 c = 0; c < nao; c++)
                            t += Vk[a * nao + c] * T[c * nao + b]
                               + Dk[c * nao + a] * U[c * nao + b];
                        out[a * nao + b] += t;
                    }
            }
            free(T);
            free(U);
        }
    }
    free(D);
    free(gam);
    free(om);
    free(dD);
}

/* Factored reverse-mode derivative (symmetric B), the half-transform form of
 * the closed forms in the header: for every density k and slab Q
 *   X = B^Q C_Lk, Y = B^Q C_Rk, P = V_k Y, R = V_k^T X,
 *   dC_Lk += B^Q P + omega_kQ Y,   dC_Rk += B^Q R + omega_kQ X,
 *   dB^Q  += gamma_kQ W_k + omega_kQ C_Lk C_Rk^T + P C_Lk^T + C_Rk R^T.
 * Slabs are processed for Q in [q0, q1) only (dB rows outside are untouched;
 * dC sums only that range), so a Q-sample can be timed.  W or V may be NULL.
 * dB is indexed by absolute Q.  Q ascending; threads split rows only. */
void jko_vjp_factored(i64 nd, i64 nao, i64 naux, i64 r, const double *B,
                      const double *CL, const double *CR, const double *W,
                      const double *V, i64 q0, i64 q1, double *dB,
                      double *dCL, double *dCR)
{
    (void)naux;
    i64 n2 = nao * nao;
    double *x = (double *)malloc(sizeof(double) * nao * r);
    double *y = (double *)malloc(sizeof(double) * nao * r);
    double *pp = (double *)malloc(sizeof(double) * nao * r);
    double *rr = (double *)malloc(sizeof(double) * nao * r);
    for (i64 e = 0; e < nd * nao * r; e++) {
        if (dCL) dCL[e] = 0.0;
        if (dCR) dCR[e] = 0.0;
    }
    if (dB)
        for (i64 q = q0; q < q1; q++)
            for (i64 e = 0; e < n2; e++)
                dB[q * n2 + e] = 0.0;
    for (i64 k = 0; k < nd; k++) {
        const double *cl = CL + k * nao * r, *cr = CR + k * nao * r;
        const double *Wk = W ? W + k * n2 : NULL, *Vk = V ? V + k * n2 : NULL;
        for (i64 q = q0; q < q1; q++) {
            const double *Bq = B + q * n2;
#pragma omp parallel for schedule(static)
            for (i64 m = 0; m < nao; m++)
                for (i64 i = 0; i < r; i++) {
                    double sx = 0.0, sy = 0.0;
                    for (i64 l = 0; l < nao; l++) {
                        sx += Bq[m * nao + l] * cl[l * r + i];
                        sy += Bq[m * nao + l] * cr[l * r + i];
                    }
                    x[m * r + i] = sx;
                    y[m * r + i] = sy;
                }
            double g = 0.0, w = 0.0;
            for (i64 m = 0; m < nao; m++)
                for (i64 i = 0; i < r; i++)
                    g += cl[m * r + i] * y[m * r + i];
            if (Wk)
                for (i64 e = 0; e < n2; e++)
                    w += Wk[e] * Bq[e];
#pragma omp parallel for schedule(static)
            for (i64 m = 0; m < nao; m++)
                for (i64 i = 0; i < r; i++) {
                    double sp = 0.0, sr = 0.0;
                    if (Vk)
                        for (i64 n = 0; n < nao; n++) {
                            sp += Vk[m * nao + n] * y[n * r + i];
                            sr += Vk[n * nao + m] * x[n * r + i];
                        }
                    pp[m * r + i] = sp;
                    rr[m * r + i] = sr;
                }
            if (dCL || dCR)
#pragma omp parallel for schedule(static)
                for (i64 m = 0; m < nao; m++)
                    for (i64 i = 0; i < r; i++) {
                        double sl = w * y[m * r + i], sr = w * x[m * r + i];
                        for (i64 n = 0; n < nao; n++) {
                            sl += Bq[m * nao + n] * pp[n * r + i];
                            sr += Bq[m * nao + n] * rr[n * r + i];
                        }
                        if (dCL)
                            dCL[(k * nao + m) * r + i] += sl;
                        if (dCR)
                            dCR[(k * nao + m) * r + i] += sr;
                    }
            if (dB)
#pragma omp parallel for schedule(static)
                for (i64 a = 0; a < nao; a++)
                    for (i64 b = 0; b < nao; b++) {
                        double v = 0.0;
                        for (i64 i = 0; i < r; i++)
                            v += w * cl[a * r + i] * cr[b * r + i]
                               + pp[a * r + i] * cl[b * r + i]
                               + cr[a * r + i] * rr[b * r + i];
                        if (Wk)
                            v += g * Wk[a * nao + b];
                        dB[q * n2 + a * nao + b] += v;
                    }
        }
    }
    free(x);
    free(y);
    free(pp);
    free(rr);
}

/* Selected entries of dB (symmetric B assumed, as the factored form uses):
 *   dB^Q_ab = sum_k gamma_kQ W_k,ab + omega_kQ D_k,ab
 *             + sum_c V_k,ac (B^Q D_k^T)_cb + sum_c D_k,ca (B^Q V_k)_cb
 * Entry e is (Q = qs[e], a = as[e], b = bs[e]). */
void jko_db_entries(i64 nd, i64 nao, i64 naux, i64 r, const double *B,
                    const double *CL, const double *CR, const double *W,
                    const double *V, i64 nent, const i64 *qs, const i64 *as,
                    const i64 *bs, double *out)
{
    (void)naux;
    i64 n2 = nao * nao;
#pragma omp parallel for schedule(dynamic, 1)
    for (i64 e = 0; e < nent; e++) {
        i64 q = qs[e], a = as[e], b = bs[e];
        const double *Bq = B + q * n2;
        double *Drow = (double *)malloc(sizeof(double) * nao); /* D_k[b][:] */
        double *Dcol = (double *)malloc(sizeof(double) * nao); /* D_k[:][a] */
        double tot = 0.0;
        for (i64 k = 0; k < nd; k++) {
            const double *cl = CL + k * nao * r, *cr = CR + k * nao * r;
            for (i64 t = 0; t < nao; t++) {
                double s1 = 0.0, s2 = 0.0;
                for (i64 i = 0; i < r; i++) {
                    s1 += cl[b * r + i] * cr[t * r + i];
                    s2 += cl[t * r + i] * cr[a * r + i];
                }
                Drow[t] = s1;
                Dcol[t] = s2;
            }
            /* gamma_kQ and omega_kQ */
            double g = 0.0, w = 0.0;
            for (i64 l = 0; l < nao; l++)
                for (i64 s = 0; s < nao; s++) {
                    double dls = 0.0;
                    for (i64 i = 0; i < r; i++)
                        dls += cl[l * r + i] * cr[s * r + i];
                    g += Bq[l * nao + s] * dls;
                    if (W)
                        w += Bq[l * nao + s] * W[k * n2 + l * nao + s];
                }
            double dab = 0.0;
            for (i64 i = 0; i < r; i++)
                dab += cl[a * r + i] * cr[b * r + i];
            double v = w * dab;
            if (W)
                v += g * W[k * n2 + a * nao + b];
            if (V) {
                const double *Vk = V + k * n2;
                for (i64 c = 0; c < nao; c++) {
                    /* (B D^T)_cb = sum_d B_cd D_bd ; (B V)_cb = sum_d B_cd V_db */
                    double t1 = 0.0, t2 = 0.0;
                    for (i64 d = 0; d < nao; d++) {
                        t1 += Bq[c * nao + d] * Drow[d];
                        t2 += Bq[c * nao + d] * Vk[d * nao + b];
                    }
                    v += Vk[a * nao + c] * t1 + Dcol[c] * t2;
                }
            }
            tot += v;
        }
        out[e] = tot;
        free(Drow);
        free(Dcol);
    }
}

/* ------------------------------------------------------- forward derivative */

/* Directional derivative of (J, K) along (dB, dC_L, dC_R), by the product
 * rule on the formulas in the header (general B):
 *   dD_k  = dC_Lk C_Rk^T + C_Lk dC_Rk^T
 *   dJ_k  = sum_Q (<dB^Q, D_k> + <B^Q, dD_k>) B^Q + gamma_kQ dB^Q
 *   dK_k  = sum_Q dB^Q D_k B^Q + B^Q dD_k B^Q + B^Q D_k dB^Q
 * Any of dB, dCL, dCR may be NULL (zero direction). */
void jko_jvp(i64 nd, i64 nao, i64 naux, i64 r, const double *B,
             const double *CL, const double *CR, const double *dB,
             const double *dCL, const double *dCR, double *dJ, double *dK)
{
    i64 n2 = nao * nao;
    double *D = (double *)malloc(sizeof(double) * nd * n2);
    double *dD = (double *)calloc(nd * n2, sizeof(double));
    double *tmp = (double *)malloc(sizeof(double) * nd * n2);
    jko_density(nd, nao, r, CL, CR, D);
    if (dCL) {
        jko_density(nd, nao, r, dCL, CR, tmp);
        for (i64 e = 0; e < nd * n2; e++)
            dD[e] += tmp[e];
    }
    if (dCR) {
        jko_density(nd, nao, r, CL, dCR, tmp);
        for (i64 e = 0; e < nd * n2; e++)
            dD[e] += tmp[e];
    }
    double *gam = (double *)malloc(sizeof(double) * nd * naux);
    double *dg = (double *)malloc(sizeof(double) * nd * naux);
    jko_project(nd, nao, naux, B, D, gam);
    jko_project(nd, nao, naux, B, dD, dg);
    if (dB) {
        double *g2 = (double *)malloc(sizeof(double) * nd * naux);
        jko_project(nd, nao, naux, dB, D, g2);
        for (i64 e = 0; e < nd * naux; e++)
            dg[e] += g2[e];
        free(g2);
    }
    jko_coulomb(nd, nao, naux, B, dg, dJ);
    if (dB) {
        jko_coulomb(nd, nao, naux, dB, gam, tmp);
        for (i64 e = 0; e < nd * n2; e++)
            dJ[e] += tmp[e];
    }
    /* dK: three literal triple products per (k, Q) */
    double *T = (double *)malloc(sizeof(double) * n2);
    for (i64 k = 0; k < nd; k++) {
        double *acc = dK + k * n2;
        for (i64 e = 0; e < n2; e++)
            acc[e] = 0.0;
        for (i64 q = 0; q < naux; q++) {
            const double *Bq = B + q * n2;
            const double *dBq = dB ? dB + q * n2 : NULL;
            for (int term = 0; term < 3; term++) {
                const double *L, *M, *Rm;
                if (term == 0) {
                    if (!dBq) continue;
                    L = dBq; M = D + k * n2; Rm = Bq;
                } else if (term == 1) {
                    L = Bq; M = dD + k * n2; Rm = Bq;
                } else {
                    if (!dBq) continue;
                    L = Bq; M = D + k * n2; Rm = dBq;
                }
#pragma omp parallel for schedule(static)
                for (i64 l = 0; l < nao; l++)
                    for (i64 n = 0; n < nao; n++) {
                        double s = 0.0;
                        for (i64 t = 0; t < nao; t++)
                            s += M[l * nao + t] * Rm[t * nao + n];
                        T[l * nao + n] = s;
                    }
#pragma omp parallel for schedule(static)
                for (i64 m = 0; m < nao; m++)
                    for (i64 n = 0; n < nao; n++) {
                        double s = 0.0;
                        for (i64 l = 0; l < nao; l++)
                            s += L[m * nao + l] * T[l * nao + n];
                        acc[m * nao + n] += s;
                    }
            }
        }
    }
    free(T);
    free(D);
    free(dD);
    free(tmp);
    free(gam);
    free(dg);
}

/* dC_Lk and dC_Rk for one density k at inputs too large for jko_vjp (symmetric
 * B assumed, as in the factored form):
 *   dC_Lk = sum_Q omega_kQ Y^Q_k + B^Q V_k Y^Q_k
 *   dC_Rk = sum_Q omega_kQ X^Q_k + B^Q V_k^T X^Q_k
 * Q-outer; each half-transform formed once per Q. */
void jko_dc_density(i64 nao, i64 naux, i64 r, const double *B,
                    const double *CLk, const double *CRk, const double *Wk,
                    const double *Vk, double *dCLk, double *dCRk)
{
    i64 n2 = nao * nao;
    double *x = (double *)malloc(sizeof(double) * nao * r);
    double *y = (double *)malloc(sizeof(double) * nao * r);
    double *p = (double *)malloc(sizeof(double) * nao * r);
    double *rr = (double *)malloc(sizeof(double) * nao * r);
    for (i64 e = 0; e < nao * r; e++) {
        dCLk[e] = 0.0;
        dCRk[e] = 0.0;
    }
    for (i64 q = 0; q < naux; q++) {
        const double *Bq = B + q * n2;
        double w = 0.0;
        if (Wk)
            for (i64 ls = 0; ls < n2; ls++)
                w += Wk[ls] * Bq[ls];
#pragma omp parallel for schedule(static)
        for (i64 m = 0; m < nao; m++)
            for (i64 i = 0; i < r; i++) {
                double sx = 0.0, sy = 0.0;
                for (i64 l = 0; l < nao; l++) {
                    sx += Bq[m * nao + l] * CLk[l * r + i];
                    sy += Bq[m * nao + l] * CRk[l * r + i];
                }
                x[m * r + i] = sx;
                y[m * r + i] = sy;
            }
#pragma omp parallel for schedule(static)
        for (i64 m = 0; m < nao; m++)
            for (i64 i = 0; i < r; i++) {
                double sp = 0.0, sr = 0.0;
                if (Vk)
                    for (i64 n = 0; n < nao; n++) {
                        sp += Vk[m * nao + n] * y[n * r + i];
                        sr += Vk[n * nao + m] * x[n * r + i];
                    }
                p[m * r + i] = sp;
                rr[m * r + i] = sr;
            }
#pragma omp parallel for schedule(static)
        for (i64 m = 0; m < nao; m++)
            for (i64 i = 0; i < r; i++) {
                double sl = w * y[m * r + i], sr = w * x[m * r + i];
                for (i64 n = 0; n < nao; n++) {
                    sl += Bq[m * nao + n] * p[n * r + i];
                    sr += Bq[m * nao + n] * rr[n * r + i];
                }
                dCLk[m * r + i] += sl;
                dCRk[m * r + i] += sr;
            }
    }
    free(x);
    free(y);
    free(p);
    free(rr);
}

/* Number of OpenMP threads the oracle runs with (for reporting). */
int jko_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

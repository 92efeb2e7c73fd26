/*
 * sanitize_check.c -- driver that runs every oracle routine on small inputs
 * held in exactly sized heap buffers, for a host build with AddressSanitizer
 * and UndefinedBehaviorSanitizer (tests/test_oracle_sanitize.py compiles it
 * with jk_oracle.c and runs it).
 *
 * TEST INFRASTRUCTURE ONLY, like jk_oracle.c: it includes nothing of the GPU
 * library.  Besides running every routine under the sanitizers it checks the
 * tiers against each other (T0 brute force through the 4-index tensor, T1
 * the plain definition, T2 the factored form, T3 single entries), the
 * reverse-mode derivative against its factored form, its single entries and
 * its per-density form, and the reverse mode against the forward mode through
 * the dot-product identity <W, dJ> + <V, dK> = <dB, tB> + <dCL, tL> + <dCR, tR>.
 * Exit status 0 and a final "ok" line when everything agrees to 1e-12.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef int64_t i64;

void jko_eri4(i64 nao, i64 naux, const double *B, double *eri);
void jko_jk_from_eri(i64 nao, const double *eri, const double *D, double *J, double *K);
void jko_density(i64 nd, i64 nao, i64 r, const double *CL, const double *CR, double *D);
void jko_project(i64 nd, i64 nao, i64 naux, const double *B, const double *A, double *g);
void jko_coulomb(i64 nd, i64 nao, i64 naux, const double *B, const double *g, double *J);
void jko_exchange(i64 nd, i64 nao, i64 naux, const double *B, const double *D, double *K);
void jko_jk_factored(i64 nd, i64 nao, i64 naux, i64 r, const double *B, const double *CL,
                     const double *CR, double *J, double *K, double *gamma_out);
void jko_jk_entries(i64 nao, i64 naux, i64 r, const double *B, const double *CL,
                    const double *CR, const double *gamma, i64 nent, const i64 *ks,
                    const i64 *ms, const i64 *ns, double *Jout, double *Kout);
void jko_vjp(i64 nd, i64 nao, i64 naux, i64 r, const double *B, const double *CL,
             const double *CR, const double *W, const double *V, double *dB, double *dCL,
             double *dCR);
void jko_vjp_factored(i64 nd, i64 nao, i64 naux, i64 r, const double *B, const double *CL,
                      const double *CR, const double *W, const double *V, i64 q0, i64 q1,
                      double *dB, double *dCL, double *dCR);
void jko_db_entries(i64 nd, i64 nao, i64 naux, i64 r, const double *B, const double *CL,
                    const double *CR, const double *W, const double *V, i64 nent,
                    const i64 *qs, const i64 *as, const i64 *bs, double *out);
void jko_jvp(i64 nd, i64 nao, i64 naux, i64 r, const double *B, const double *CL,
             const double *CR, const double *dB, const double *dCL, const double *dCR,
             double *dJ, double *dK);
void jko_dc_density(i64 nao, i64 naux, i64 r, const double *B, const double *CLk,
                    const double *CRk, const double *Wk, const double *Vk, double *dCLk,
                    double *dCRk);

static uint64_t state = 0x9E3779B97F4A7C15ull;

/* uniform in [-1, 1) from a 64-bit linear congruential generator */
static double uni(void)
{
    state = state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(state >> 11) * 0x1p-52 - 1.0;
}

static double *vec(i64 n, int fill)
{
    double *p = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!p) {
        fprintf(stderr, "out of memory\n");
        exit(2);
    }
    for (i64 i = 0; i < n; i++)
        p[i] = fill ? uni() : 0.0;
    return p;
}

static int failures = 0;

/* normwise relative difference, reported against tol */
static void agree(const char *what, const double *a, const double *b, i64 n, double tol)
{
    double d = 0.0, m = 0.0;
    for (i64 i = 0; i < n; i++) {
        d = fmax(d, fabs(a[i] - b[i]));
        m = fmax(m, fabs(b[i]));
    }
    const double rel = m > 0.0 ? d / m : d;
    printf("%-44s %.2e\n", what, rel);
    if (!(rel <= tol)) {
        printf("  MISMATCH (tolerance %.0e)\n", tol);
        failures++;
    }
}

int main(void)
{
    const i64 nao = 7, naux = 5, nd = 2, r = 3, n2 = nao * nao;
    const double tol = 1e-12;
    double *B = vec(naux * n2, 1);
    for (i64 q = 0; q < naux; q++) /* symmetric slabs */
        for (i64 m = 0; m < nao; m++)
            for (i64 n = 0; n < m; n++)
                B[(q * nao + m) * nao + n] = B[(q * nao + n) * nao + m];
    double *CL = vec(nd * nao * r, 1), *CR = vec(nd * nao * r, 1);
    double *W = vec(nd * n2, 1), *V = vec(nd * n2, 1);

    /* T0 through the 4-index tensor, one density at a time */
    double *eri = vec(n2 * n2, 0), *D = vec(nd * n2, 0);
    double *J0 = vec(nd * n2, 0), *K0 = vec(nd * n2, 0);
    jko_eri4(nao, naux, B, eri);
    jko_density(nd, nao, r, CL, CR, D);
    for (i64 k = 0; k < nd; k++)
        jko_jk_from_eri(nao, eri, D + k * n2, J0 + k * n2, K0 + k * n2);

    /* T1: explicit D and literal products */
    double *g = vec(nd * naux, 0), *J1 = vec(nd * n2, 0), *K1 = vec(nd * n2, 0);
    jko_project(nd, nao, naux, B, D, g);
    jko_coulomb(nd, nao, naux, B, g, J1);
    jko_exchange(nd, nao, naux, B, D, K1);
    agree("J: plain definition vs 4-index tensor", J1, J0, nd * n2, tol);
    agree("K: plain definition vs 4-index tensor", K1, K0, nd * n2, tol);

    /* T2: factored */
    double *J2 = vec(nd * n2, 0), *K2 = vec(nd * n2, 0), *g2 = vec(nd * naux, 0);
    jko_jk_factored(nd, nao, naux, r, B, CL, CR, J2, K2, g2);
    agree("J: factored vs plain", J2, J1, nd * n2, tol);
    agree("K: factored vs plain", K2, K1, nd * n2, tol);
    agree("gamma: factored vs projection", g2, g, nd * naux, tol);

    /* T3: every entry one by one */
    const i64 nent = nd * n2;
    i64 *ks = (i64 *)malloc(sizeof(i64) * nent), *ms = (i64 *)malloc(sizeof(i64) * nent);
    i64 *ns = (i64 *)malloc(sizeof(i64) * nent);
    for (i64 e = 0; e < nent; e++) {
        ks[e] = e / n2;
        ms[e] = (e % n2) / nao;
        ns[e] = e % nao;
    }
    double *Je = vec(nent, 0), *Ke = vec(nent, 0);
    jko_jk_entries(nao, naux, r, B, CL, CR, g, nent, ks, ms, ns, Je, Ke);
    agree("J: single entries vs plain", Je, J1, nent, tol);
    agree("K: single entries vs plain", Ke, K1, nent, tol);

    /* reverse mode: literal, factored over all slabs and over two ranges */
    double *dB = vec(naux * n2, 0), *dCL = vec(nd * nao * r, 0), *dCR = vec(nd * nao * r, 0);
    jko_vjp(nd, nao, naux, r, B, CL, CR, W, V, dB, dCL, dCR);
    double *fB = vec(naux * n2, 0), *fL = vec(nd * nao * r, 0), *fR = vec(nd * nao * r, 0);
    jko_vjp_factored(nd, nao, naux, r, B, CL, CR, W, V, 0, naux, fB, fL, fR);
    agree("dB: factored vs literal", fB, dB, naux * n2, tol);
    agree("dCL: factored vs literal", fL, dCL, nd * nao * r, tol);
    agree("dCR: factored vs literal", fR, dCR, nd * nao * r, tol);
    double *hB = vec(naux * n2, 0), *hL = vec(nd * nao * r, 0), *hR = vec(nd * nao * r, 0);
    double *hL2 = vec(nd * nao * r, 0), *hR2 = vec(nd * nao * r, 0);
    jko_vjp_factored(nd, nao, naux, r, B, CL, CR, W, V, 0, 2, hB, hL, hR);
    jko_vjp_factored(nd, nao, naux, r, B, CL, CR, W, V, 2, naux, hB, hL2, hR2);
    for (i64 i = 0; i < nd * nao * r; i++) {
        hL[i] += hL2[i];
        hR[i] += hR2[i];
    }
    agree("dB: two slab ranges vs literal", hB, dB, naux * n2, tol);
    agree("dCL: two slab ranges vs literal", hL, dCL, nd * nao * r, tol);

    /* single entries of dB */
    const i64 nb = naux * n2;
    i64 *qs = (i64 *)malloc(sizeof(i64) * nb), *as = (i64 *)malloc(sizeof(i64) * nb);
    i64 *bs = (i64 *)malloc(sizeof(i64) * nb);
    for (i64 e = 0; e < nb; e++) {
        qs[e] = e / n2;
        as[e] = (e % n2) / nao;
        bs[e] = e % nao;
    }
    double *dBe = vec(nb, 0);
    jko_db_entries(nd, nao, naux, r, B, CL, CR, W, V, nb, qs, as, bs, dBe);
    agree("dB: single entries vs literal", dBe, dB, nb, tol);

    /* per-density gradient of C */
    double *cL = vec(nao * r, 0), *cR = vec(nao * r, 0);
    jko_dc_density(nao, naux, r, B, CL + nao * r, CR + nao * r, W + n2, V + n2, cL, cR);
    agree("dCL of density 1: per-density vs literal", cL, dCL + nao * r, nao * r, tol);
    agree("dCR of density 1: per-density vs literal", cR, dCR + nao * r, nao * r, tol);

    /* forward mode against reverse mode */
    double *tB = vec(naux * n2, 1), *tL = vec(nd * nao * r, 1), *tR = vec(nd * nao * r, 1);
    double *dJ = vec(nd * n2, 0), *dK = vec(nd * n2, 0);
    jko_jvp(nd, nao, naux, r, B, CL, CR, tB, tL, tR, dJ, dK);
    double lhs = 0.0, rhs = 0.0;
    for (i64 i = 0; i < nd * n2; i++)
        lhs += W[i] * dJ[i] + V[i] * dK[i];
    for (i64 i = 0; i < naux * n2; i++)
        rhs += dB[i] * tB[i];
    for (i64 i = 0; i < nd * nao * r; i++)
        rhs += dCL[i] * tL[i] + dCR[i] * tR[i];
    agree("<W,dJ>+<V,dK> vs <dB,tB>+<dC,tC>", &lhs, &rhs, 1, tol);

    free(B); free(CL); free(CR); free(W); free(V); free(eri); free(D); free(J0); free(K0);
    free(g); free(J1); free(K1); free(J2); free(K2); free(g2); free(ks); free(ms); free(ns);
    free(Je); free(Ke); free(dB); free(dCL); free(dCR); free(fB); free(fL); free(fR);
    free(hB); free(hL); free(hR); free(hL2); free(hR2); free(qs); free(as); free(bs); free(dBe);
    free(cL); free(cR); free(tB); free(tL); free(tR); free(dJ); free(dK);
    if (failures) {
        printf("%d mismatches\n", failures);
        return 1;
    }
    printf("ok\n");
    return 0;
}

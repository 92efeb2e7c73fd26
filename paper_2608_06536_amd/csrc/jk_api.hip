// jk_api.hip -- the C ABI (include/jk.h): validation, workspace plan, launch
// sequence.  Host code only; kernels live in jk_fp64.hip and friends.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include "../../include/jk.h"
#include "jk_kernels.hpp"

namespace {

typedef int64_t i64;

constexpr size_t kAlign = 256;
constexpr i64 kMaxNao = 16384;          // keeps every tile index in 32 bits
constexpr i64 kMaxCols = 1 << 20;       // 2 * ndens * rank
constexpr size_t kChunkBudget = (size_t)256 << 20;   // X/Y chunk workspace target

inline size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

struct Carve {
    size_t off = 0;
    size_t take(size_t bytes)
    {
        size_t o = off;
        off = align_up(off + bytes);
        return o;
    }
};

bool valid_problem(const jk_problem *p)
{
    if (!p)
        return false;
    if (p->nao < 1 || p->nao > kMaxNao || p->naux < 1 || p->ndens < 1 || p->rank < 1)
        return false;
    if (p->rank > p->nao)
        return false;
    if (2 * p->ndens * p->rank > kMaxCols)
        return false;
    if (p->naux > (i64)1 << 28)
        return false;
    if (p->precision != JK_FP64 && p->precision != JK_MIXED)
        return false;
    if (p->flags < 0 || p->flags > (JK_WANT_J | JK_WANT_K))
        return false;
    if (p->reserved != 0)
        return false;
    if (p->precision == JK_MIXED && p->nslice != 0 && (p->nslice < 2 || p->nslice > 5))
        return false;
    return true;
}

inline int want(const jk_problem *p) { return p->flags == 0 ? (JK_WANT_J | JK_WANT_K) : p->flags; }

// Slabs per chunk of the half-transform workspace.
int chunk_slabs(const jk_problem *p)
{
    size_t per = 2 * (size_t)p->nao * (size_t)(p->ndens * p->rank) * sizeof(double);
    i64 qc = (i64)(kChunkBudget / (per ? per : 1));
    if (qc < 1)
        qc = 1;
    if (qc > p->naux)
        qc = p->naux;
    return (int)qc;
}

struct FwdPlan {
    int qc, ldw, npb, plen, ndp, nsplit;
    size_t o_cc, o_d, o_part, o_g, o_x, o_y, o_kp, total;
};

FwdPlan plan_forward(const jk_problem *p)
{
    FwdPlan f;
    const i64 nao = p->nao, nd = p->ndens, r = p->rank, R = nd * r;
    const i64 npos = nao * nao;
    f.qc = chunk_slabs(p);
    f.ldw = (int)(f.qc * r);
    f.ndp = (int)(((nd + 7) / 8) * 8);
    f.npb = jk::project_nblocks(npos, (int)p->naux, (int)nd, &f.plen);
    Carve c;
    f.o_cc = c.take(sizeof(double) * nao * 2 * R);
    f.o_d = c.take(sizeof(double) * nd * npos);
    f.o_part = c.take(sizeof(double) * (size_t)f.npb * p->naux * f.ndp);
    f.o_g = c.take(sizeof(double) * nd * p->naux);
    f.o_x = c.take(sizeof(double) * nd * nao * (size_t)f.ldw);
    f.o_y = c.take(sizeof(double) * nd * nao * (size_t)f.ldw);
    f.nsplit = jk::exchange_nsplit((int)nao, (int)nd, f.ldw);
    f.o_kp = c.take(f.nsplit > 1 ? sizeof(double) * (size_t)f.nsplit * nd * npos : 0);
    f.total = c.off;
    return f;
}

// Slabs per chunk of the derivative: X, Y, P, R of one chunk in the budget.
int chunk_slabs_vjp(const jk_problem *p)
{
    size_t per = 4 * (size_t)p->nao * (size_t)(p->ndens * p->rank) * sizeof(double);
    i64 qc = (i64)(kChunkBudget / (per ? per : 1));
    if (qc < 1)
        qc = 1;
    if (qc > p->naux)
        qc = p->naux;
    return (int)qc;
}

struct VjpPlan {
    int qc, ldw, npb, plen, ndp, nsplit_c;
    size_t o_cc, o_d, o_part, o_g, o_om, o_omx, o_x, o_y, o_p, o_r, o_dcp, total;
};

VjpPlan plan_vjp(const jk_problem *p)
{
    VjpPlan f;
    const i64 nao = p->nao, nd = p->ndens, r = p->rank, R = nd * r, naux = p->naux;
    const i64 npos = nao * nao;
    f.qc = chunk_slabs_vjp(p);
    f.ldw = (int)(f.qc * r);
    f.ndp = (int)(((nd + 7) / 8) * 8);
    f.npb = jk::project_nblocks(npos, (int)naux, (int)nd, &f.plen);
    f.nsplit_c = jk::vjp_stage_c_nsplit((int)nao, (int)R, f.qc);
    Carve c;
    f.o_cc = c.take(sizeof(double) * nao * 2 * R);
    f.o_d = c.take(sizeof(double) * nd * npos);
    f.o_part = c.take(sizeof(double) * (size_t)f.npb * naux * f.ndp);
    f.o_g = c.take(sizeof(double) * nd * naux);
    f.o_om = c.take(sizeof(double) * nd * naux);
    f.o_omx = c.take(sizeof(double) * naux * R);
    f.o_x = c.take(sizeof(double) * nd * nao * (size_t)f.ldw);
    f.o_y = c.take(sizeof(double) * nd * nao * (size_t)f.ldw);
    f.o_p = c.take(sizeof(double) * (size_t)f.qc * nao * R);
    f.o_r = c.take(sizeof(double) * (size_t)f.qc * nao * R);
    f.o_dcp = c.take(sizeof(double) * (size_t)f.nsplit_c * nao * 2 * R);
    f.total = c.off;
    return f;
}

#define JK_TRY(expr)                                                                               \
    do {                                                                                           \
        hipError_t _e = (expr);                                                                    \
        if (_e != hipSuccess)                                                                      \
            return JK_EHIP;                                                                        \
    } while (0)

jk_status build_fp64(const jk_problem *p, const double *B, const double *CL, const double *CR,
                     double *J, double *K, char *ws, hipStream_t s)
{
    const FwdPlan f = plan_forward(p);
    const int nao = (int)p->nao, naux = (int)p->naux, nd = (int)p->ndens, r = (int)p->rank;
    const i64 npos = (i64)nao * nao;
    const int w = want(p);
    double *Cc = (double *)(ws + f.o_cc);
    double *D = (double *)(ws + f.o_d);
    double *part = (double *)(ws + f.o_part);
    double *g = (double *)(ws + f.o_g);
    double *Xw = (double *)(ws + f.o_x);
    double *Yw = (double *)(ws + f.o_y);

    if (w & JK_WANT_J) {
        // gamma_kQ = <D_k, B^Q> in FP64, then J_k = sum_Q gamma_kQ B^Q.
        JK_TRY(jk::launch_density(CL, CR, D, nao, nd, r, s));
        JK_TRY(jk::launch_project(B, D, part, g, naux, nd, npos, s));
        JK_TRY(jk::launch_coulomb(B, g, J, naux, nd, npos, s));
    }
    if (w & JK_WANT_K) {
        // K accumulates over Q-chunks in nsplit partial buffers (or in K
        // itself when nsplit == 1), summed in fixed order at the end.
        double *Kp = f.nsplit > 1 ? (double *)(ws + f.o_kp) : K;
        JK_TRY(jk::launch_pack_c(CL, CR, Cc, nao, nd, r, s));
        for (int q0 = 0; q0 < naux; q0 += f.qc) {
            int nq = (naux - q0) < f.qc ? (naux - q0) : f.qc;
            JK_TRY(jk::launch_half_transform(B, Cc, Xw, Yw, nao, nd, r, q0, nq, f.ldw, s));
            JK_TRY(jk::launch_exchange(Xw, Yw, Kp, nao, nd, nq * r, f.ldw, f.nsplit, q0 > 0, s));
        }
        if (f.nsplit > 1)
            JK_TRY(jk::launch_sum_splits(Kp, K, (i64)nd * npos, f.nsplit, s));
    }
    return JK_OK;
}

jk_status vjp_fp64(const jk_problem *p, const double *B, const double *CL, const double *CR,
                   const double *W, const double *V, double *dB, double *dCL, double *dCR, char *ws,
                   hipStream_t s)
{
    const VjpPlan f = plan_vjp(p);
    const int nao = (int)p->nao, naux = (int)p->naux, nd = (int)p->ndens, r = (int)p->rank;
    const int R = nd * r;
    const i64 npos = (i64)nao * nao;
    const int has_w = W != nullptr, has_v = V != nullptr;
    const bool want_db = dB != nullptr, want_dc = dCL != nullptr;
    double *Cc = (double *)(ws + f.o_cc);
    double *D = (double *)(ws + f.o_d);
    double *part = (double *)(ws + f.o_part);
    double *g = (double *)(ws + f.o_g);
    double *om = (double *)(ws + f.o_om);
    double *omx = (double *)(ws + f.o_omx);
    double *Xw = (double *)(ws + f.o_x);
    double *Yw = (double *)(ws + f.o_y);
    double *Pq = (double *)(ws + f.o_p);
    double *Rq = (double *)(ws + f.o_r);
    double *dCp = (double *)(ws + f.o_dcp);

    JK_TRY(jk::launch_pack_c(CL, CR, Cc, nao, nd, r, s));
    if (has_w) {
        // omega_kQ = <W_k, B^Q>; gamma_kQ = <D_k, B^Q> for the gamma W term of dB.
        JK_TRY(jk::launch_project(B, W, part, om, naux, nd, npos, s));
        JK_TRY(jk::launch_omega_expand(om, omx, naux, nd, r, s));
        if (want_db) {
            JK_TRY(jk::launch_density(CL, CR, D, nao, nd, r, s));
            JK_TRY(jk::launch_project(B, D, part, g, naux, nd, npos, s));
        }
    }
    for (int q0 = 0; q0 < naux; q0 += f.qc) {
        const int nq = (naux - q0) < f.qc ? (naux - q0) : f.qc;
        if (has_v) {
            JK_TRY(jk::launch_half_transform(B, Cc, Xw, Yw, nao, nd, r, q0, nq, f.ldw, s));
            JK_TRY(jk::launch_vjp_stage_b(V, Xw, Yw, Pq, Rq, nao, nd, r, nq * r, f.ldw, s));
        }
        if (want_dc)
            JK_TRY(jk::launch_vjp_stage_c(B, Pq, Rq, omx, Cc, dCp, nao, R, q0, nq, f.nsplit_c, has_v,
                                          has_w, q0 > 0, s));
        if (want_db)
            JK_TRY(jk::launch_vjp_stage_d(Pq, Rq, Cc, omx, g, W, dB, nao, nd, r, naux, q0, nq, has_v,
                                          has_w, s));
    }
    if (want_dc)
        JK_TRY(jk::launch_vjp_dc_finish(dCp, dCL, dCR, nao, nd, r, f.nsplit_c, s));
    return JK_OK;
}

} // namespace

extern "C" {

size_t jk_workspace_bytes(const jk_problem *p)
{
    if (!valid_problem(p))
        return 0;
    size_t a = plan_forward(p).total, b = plan_vjp(p).total;
    return a > b ? a : b;
}

jk_status jk_build(const jk_problem *p, const double *B, const double *CL, const double *CR,
                   double *J, double *K, void *ws, size_t ws_bytes, void *stream)
{
    if (!valid_problem(p))
        return JK_EINVAL;
    const int w = want(p);
    if (!B || !CL || !CR || !ws)
        return JK_EINVAL;
    if ((w & JK_WANT_J) && !J)
        return JK_EINVAL;
    if ((w & JK_WANT_K) && !K)
        return JK_EINVAL;
    if (((uintptr_t)ws) % kAlign)
        return JK_EINVAL;
    if (ws_bytes < jk_workspace_bytes(p))
        return JK_EWORKSPACE;
    if (p->precision != JK_FP64)
        return JK_EUNSUPPORTED;
    return build_fp64(p, B, CL, CR, J, K, (char *)ws, (hipStream_t)stream);
}

size_t jk_batched_workspace_bytes(int32_t nprob, const jk_problem *p)
{
    if (nprob < 1 || !p)
        return 0;
    size_t mx = 0;
    for (int32_t g = 0; g < nprob; g++) {
        size_t b = jk_workspace_bytes(&p[g]);
        if (b == 0)
            return 0;
        if (b > mx)
            mx = b;
    }
    return mx;
}

jk_status jk_build_batched(int32_t nprob, const jk_problem *p, const double *const *B,
                           const double *const *CL, const double *const *CR, double *const *J,
                           double *const *K, void *ws, size_t ws_bytes, void *stream)
{
    if (nprob < 1 || !p || !B || !CL || !CR || !J || !K)
        return JK_EINVAL;
    for (int32_t g = 0; g < nprob; g++) {
        if (!valid_problem(&p[g]))
            return JK_EINVAL;
        if (p[g].precision != p[0].precision || p[g].flags != p[0].flags)
            return JK_EINVAL;
        const int w = want(&p[g]);
        if (!B[g] || !CL[g] || !CR[g] || ((w & JK_WANT_J) && !J[g]) || ((w & JK_WANT_K) && !K[g]))
            return JK_EINVAL;
    }
    if (!ws || ((uintptr_t)ws) % kAlign)
        return JK_EINVAL;
    if (ws_bytes < jk_batched_workspace_bytes(nprob, p))
        return JK_EWORKSPACE;
    if (p[0].precision != JK_FP64)
        return JK_EUNSUPPORTED;
    for (int32_t g = 0; g < nprob; g++) {
        jk_status st = build_fp64(&p[g], B[g], CL[g], CR[g], J[g], K[g], (char *)ws,
                                  (hipStream_t)stream);
        if (st != JK_OK)
            return st;
    }
    return JK_OK;
}

jk_status jk_vjp(const jk_problem *p, const double *B, const double *CL, const double *CR,
                 const double *Jbar, const double *Kbar, double *dB, double *dCL, double *dCR,
                 void *ws, size_t ws_bytes, void *stream)
{
    if (!valid_problem(p))
        return JK_EINVAL;
    if (!B || !CL || !CR || !ws || ((uintptr_t)ws) % kAlign)
        return JK_EINVAL;
    if ((dCL == nullptr) != (dCR == nullptr))
        return JK_EINVAL;
    if (ws_bytes < jk_workspace_bytes(p))
        return JK_EWORKSPACE;
    if (p->precision != JK_FP64)
        return JK_EUNSUPPORTED;
    if (!dB && !dCL)
        return JK_OK;
    return vjp_fp64(p, B, CL, CR, Jbar, Kbar, dB, dCL, dCR, (char *)ws, (hipStream_t)stream);
}

const char *jk_status_str(jk_status s)
{
    switch (s) {
    case JK_OK: return "ok";
    case JK_EINVAL: return "invalid argument";
    case JK_EWORKSPACE: return "workspace too small";
    case JK_EUNSUPPORTED: return "unsupported combination";
    case JK_EHIP: return "HIP launch or runtime failure";
    }
    return "unknown status";
}

} // extern "C"

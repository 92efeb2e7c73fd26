// jk_laplace.hip -- Laplace pseudo-density driver (include/jk_laplace.h).
//
// The paper, Sec. 2.2, Eq. (laplace): an orbital-energy denominator is a
// Laplace integral discretized by a short exponential sum, and the
// exponential factorizes over the orbital indices, so a denominator-weighted
// density is a set of ordinary densities built from energy-scaled
// coefficients, each one J/K build (Sec. 2.3).
//
//   quadrature   host: minimax rule for the relative error of 1/x
//   factors      device: out = coef_k C diag(exp(s alpha_k e)) [X_m^T]
//   build        device: transition pseudo-density factors into the
//                workspace, then the ordinary J/K build on them
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "../../include/jk_laplace.h"
#include "f64_core.hpp"
#include "jk_kernels.hpp"
#include "laplace_rule.hpp"

namespace {

typedef int64_t i64;
constexpr int kMaxPts = JK_LAPLACE_MAX_POINTS;

// ===================================================================== rules
// Rules are cached per (points, range ratio): a fit takes 0.1..5 s.
struct RuleKey {
    int n;
    double R;
    bool operator<(const RuleKey &o) const { return n != o.n ? n < o.n : R < o.R; }
};
struct RuleEntry {
    jk_rule::Rule rule;
    double err = 0.0;
    bool level = false;
};
std::mutex g_rule_mu;
std::map<RuleKey, RuleEntry> g_rules;

// ==================================================================== kernels
struct LapPts {
    double alpha[kMaxPts];
    double coef[kMaxPts];
};

// out[k][m][t] = coef_k C[t] exp(s alpha_k e[t % norb]) for t < nao * norb.
__global__ void __launch_bounds__(256) k_laplace_scale(const double *__restrict__ C,
                                                       const double *__restrict__ e,
                                                       double *__restrict__ out, i64 n, int norb,
                                                       int nvec, double scale, LapPts pts)
{
    const int k = blockIdx.y;
    const double sa = scale * pts.alpha[k], c = pts.coef[k];
    for (i64 t = (i64)blockIdx.x * 256 + threadIdx.x; t < n; t += (i64)gridDim.x * 256) {
        const double v = c * C[t] * exp(sa * e[t % norb]);
        for (int m = 0; m < nvec; m++)
            out[((i64)k * nvec + m) * n + t] = v;
    }
}

// B operand of the fold: element (i, a) = X[i][a] exp(sa e[a]).
struct OpScaledRow {
    static constexpr bool kContig = true;
    static constexpr int NRAW = 2;
    const double *p;
    const double *e;
    i64 ld;
    int ni, nk;
    double sa;
    __device__ __forceinline__ void fetch(int i, int k, double *raw) const
    {
        const int ic = i < ni ? i : ni - 1, kc = k < nk ? k : nk - 1;
        raw[0] = p[(i64)ic * ld + kc];
        raw[1] = e[kc];
    }
    __device__ __forceinline__ double finish(int i, int k, const double *raw) const
    {
        return (i < ni && k < nk) ? raw[0] * exp(sa * raw[1]) : 0.0;
    }
};

typedef jk::Tile<64, 64, 32, 32, 16> TileFold;

// out[k][m] = coef_k C diag(exp(s alpha_k e)) X_m^T: one 64 x 64 output tile
// per workgroup; blockIdx.x = (k * nvec + m) * tiles + tile.
__global__ void __launch_bounds__(256) k_laplace_fold(const double *__restrict__ C,
                                                      const double *__restrict__ e,
                                                      const double *__restrict__ X,
                                                      double *__restrict__ out, int nao, int norb,
                                                      int rank, int nvec, double scale, LapPts pts)
{
    __shared__ double lds[TileFold::LDS_DOUBLES];
    const int tn = (rank + 63) / 64, tiles = ((nao + 63) / 64) * tn;
    const int km = blockIdx.x / tiles, t = blockIdx.x % tiles;
    const int k = km / nvec, m = km % nvec;
    const int m0 = (t / tn) * 64, n0 = (t % tn) * 64;
    jk::OpKC A{C, (i64)norb, nao, norb};
    OpScaledRow Bop{X + (i64)m * rank * norb, e, (i64)norb, rank, norb, scale * pts.alpha[k]};
    jk::Acc<TileFold> acc;
    acc.zero();
    jk::tile_gemm<TileFold>(A, Bop, m0, n0, 0, norb, lds, acc);
    const double c = pts.coef[k];
    double *o = out + (i64)km * nao * rank;
    jk::tile_foreach(acc, m0, n0, [&](int row, int col, double v) {
        if (row < nao && col < rank)
            o[(i64)row * rank + col] = c * v;
    });
}

constexpr i64 kMaxDim = 16384;

bool valid_factor_args(i64 nao, i64 norb, i64 rank, i64 nvec, int32_t npts)
{
    if (nao < 1 || nao > kMaxDim || norb < 1 || norb > kMaxDim || rank < 1 || rank > kMaxDim)
        return false;
    if (nvec < 1 || npts < 1 || npts > kMaxPts)
        return false;
    if (nvec > ((i64)1 << 40) / ((i64)npts * nao * rank))
        return false;
    return true;
}

jk_status launch_factors(i64 nao, i64 norb, i64 rank, i64 nvec, int32_t npts, const double *C,
                         const double *e, const double *X, const LapPts &pts, double scale,
                         double *out, hipStream_t s)
{
    if (X == nullptr) {
        const i64 n = nao * norb;
        i64 blocks = (n + 255) / 256;
        if (blocks > 4096)
            blocks = 4096;
        jk::ProfScope ps_("laplace_scale", s);
        hipLaunchKernelGGL(k_laplace_scale, dim3((unsigned)blocks, (unsigned)npts), dim3(256), 0, s,
                           C, e, out, n, (int)norb, (int)nvec, scale, pts);
    } else {
        const i64 tiles = ((nao + 63) / 64) * ((rank + 63) / 64);
        const i64 grid = tiles * npts * nvec;
        if (grid > 0x7fffffff)
            return JK_EINVAL;
        jk::ProfScope ps_("laplace_fold", s);
        hipLaunchKernelGGL(k_laplace_fold, dim3((unsigned)grid), dim3(256), 0, s, C, e, X, out,
                           (int)nao, (int)norb, (int)rank, (int)nvec, scale, pts);
    }
    return hipGetLastError() == hipSuccess ? JK_OK : JK_EHIP;
}

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

bool make_build_problem(const jk_laplace_problem *p, jk_problem &q)
{
    if (!p || p->npts < 1 || p->npts > kMaxPts || p->nocc < 1 || p->nocc > p->nao ||
        p->nvir < 1 || p->nvir > kMaxDim || p->nvec < 1)
        return false;
    if (p->nvec > ((i64)1 << 30) / p->npts)
        return false;
    q.nao = p->nao;
    q.naux = p->naux;
    q.ndens = (i64)p->npts * p->nvec;
    q.rank = p->nocc;
    q.precision = p->precision;
    q.flags = p->flags;
    q.nslice = p->nslice;
    q.reserved = 0;
    return jk_workspace_bytes(&q) != 0;
}

size_t factor_bytes(const jk_problem &q) { return align_up((size_t)q.ndens * q.nao * q.rank * sizeof(double)); }

} // namespace

extern "C" {

static jk_status jk_laplace_quadrature_impl(int32_t npts, double x_min, double x_max, double *w, double *alpha,
                                double *max_rel_err, int32_t *is_minimax)
{
    if (npts < 1 || npts > kMaxPts || !w || !alpha)
        return JK_EINVAL;
    if (!(x_min > 0.0) || !(x_max >= x_min) || !std::isfinite(x_max) || x_max / x_min > 1e9)
        return JK_EINVAL;
    const double R = std::max(x_max / x_min, 2.0);
    RuleEntry ent;
    {
        std::lock_guard<std::mutex> lk(g_rule_mu);
        auto it = g_rules.find({npts, R});
        if (it != g_rules.end()) {
            ent = it->second;
        } else {
            ent.rule = jk_rule::minimax(npts, R, ent.err, ent.level);
            g_rules[{npts, R}] = ent;
        }
    }
    for (int k = 0; k < npts; k++) {
        w[k] = std::exp(ent.rule.u[k]) / x_min;
        alpha[k] = std::exp(ent.rule.v[k]) / x_min;
    }
    if (max_rel_err)
        *max_rel_err = ent.err;
    if (is_minimax)
        *is_minimax = ent.level ? 1 : 0;
    return JK_OK;
}

jk_status jk_laplace_quadrature(int32_t npts, double x_min, double x_max, double *w, double *alpha,
                                double *max_rel_err, int32_t *is_minimax)
{
    try {
        return jk_laplace_quadrature_impl(npts, x_min, x_max, w, alpha, max_rel_err, is_minimax);
    } catch (...) {
        return JK_ENOMEM;
    }
}

jk_status jk_laplace_factors(int64_t nao, int64_t norb, int64_t rank, int64_t nvec, int32_t npts,
                             const double *C, const double *e, const double *X,
                             const double *alpha, const double *coef, double scale, double *out,
                             void *stream)
{
    if (!valid_factor_args(nao, norb, rank, nvec, npts))
        return JK_EINVAL;
    if (!C || !e || !alpha || !coef || !out || !std::isfinite(scale))
        return JK_EINVAL;
    if (!X && rank != norb)
        return JK_EINVAL;
    LapPts pts{};
    for (int k = 0; k < npts; k++) {
        if (!std::isfinite(alpha[k]) || !std::isfinite(coef[k]))
            return JK_EINVAL;
        pts.alpha[k] = alpha[k];
        pts.coef[k] = coef[k];
    }
    return launch_factors(nao, norb, rank, nvec, npts, C, e, X, pts, scale, out,
                          (hipStream_t)stream);
}

size_t jk_laplace_workspace_bytes(const jk_laplace_problem *p)
{
    jk_problem q;
    if (!make_build_problem(p, q))
        return 0;
    return 2 * factor_bytes(q) + jk_workspace_bytes(&q);
}

static jk_status jk_laplace_build_impl(const jk_laplace_problem *p, const double *B, const double *Cocc,
                           const double *e_occ, const double *Cvir, const double *e_vir,
                           const double *X, const double *w, const double *alpha, double shift,
                           double *J, double *K, void *ws, size_t ws_bytes, void *stream)
{
    jk_problem q;
    if (!make_build_problem(p, q))
        return JK_EINVAL;
    const int want = q.flags == 0 ? (JK_WANT_J | JK_WANT_K) : q.flags;
    if (!B || !Cocc || !e_occ || !Cvir || !e_vir || !X || !w || !alpha || !ws)
        return JK_EINVAL;
    if (((want & JK_WANT_J) && !J) || ((want & JK_WANT_K) && !K))
        return JK_EINVAL;
    if (((uintptr_t)ws) % kAlign || !std::isfinite(shift))
        return JK_EINVAL;
    if (ws_bytes < jk_laplace_workspace_bytes(p))
        return JK_EWORKSPACE;
    LapPts left{}, right{};
    for (int k = 0; k < p->npts; k++) {
        if (!std::isfinite(w[k]) || !std::isfinite(alpha[k]))
            return JK_EINVAL;
        left.alpha[k] = right.alpha[k] = alpha[k];
        left.coef[k] = w[k] * std::exp(-alpha[k] * shift);
        right.coef[k] = 1.0;
    }
    const size_t fb = factor_bytes(q);
    double *CL = (double *)ws;
    double *CR = (double *)((char *)ws + fb);
    void *rest = (char *)ws + 2 * fb;
    hipStream_t s = (hipStream_t)stream;
    jk_status st = launch_factors(p->nao, p->nocc, p->nocc, p->nvec, p->npts, Cocc, e_occ, nullptr,
                                  left, +1.0, CL, s);
    if (st != JK_OK)
        return st;
    st = launch_factors(p->nao, p->nvir, p->nocc, p->nvec, p->npts, Cvir, e_vir, X, right, -1.0, CR,
                        s);
    if (st != JK_OK)
        return st;
    return jk_build(&q, B, CL, CR, J, K, rest, ws_bytes - 2 * fb, stream);
}

jk_status jk_laplace_build(const jk_laplace_problem *p, const double *B, const double *Cocc,
                           const double *e_occ, const double *Cvir, const double *e_vir,
                           const double *X, const double *w, const double *alpha, double shift,
                           double *J, double *K, void *ws, size_t ws_bytes, void *stream)
{
    try {
        return jk_laplace_build_impl(p, B, Cocc, e_occ, Cvir, e_vir, X, w, alpha, shift, J, K, ws, ws_bytes, stream);
    } catch (...) {
        return JK_ENOMEM;
    }
}

} // extern "C"

// jk_api.hip -- the C ABI (include/jk.h): validation, workspace plan, launch
// sequence.  Host code only; kernels live in jk_fp64.hip and friends.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>
#include <cstring>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/jk.h"
#include "jk_batched.hpp"
#include "jk_kernels.hpp"
#include "coulomb_upper.hpp"
#include "jk_tiles.hpp"
#include "jk_tune.hpp"

// Device memory of jk_build_noalloc (jk.h): every kernel buffer of that entry
// point lives here instead of in a caller's workspace.  One copy per device,
// held until the process ends.  Host code never passes this name to a kernel
// or a copy: it uses the device address that scratch_address() looks up.
constexpr size_t kNoAllocScratchBytes = (size_t)256 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

typedef int64_t i64;

constexpr size_t kAlign = 256;
constexpr i64 kMaxNao = 16384;          // keeps every tile index in 32 bits
constexpr i64 kMaxCols = 1 << 20;       // 2 * ndens * rank
// Chunk workspace target (X/Y of the build, X/Y and slab blocks of the
// derivative): fewer, longer launches; 1 GB is small next to HBM3E.
constexpr size_t kChunkBudget = (size_t)1 << 30;
// Members of a batched build each own their chunk buffers.  FP64 members
// take the single build's 1 GB target (fewer chunk steps, each launch over
// every member's chunk; 355 against 377 ms with 256 MB on the 64-geometry
// batch); JK_MIXED members, whose chunk buffers also hold digit planes and a
// second X/Y buffer, take 256 MB.
constexpr size_t kChunkBudgetBatched = (size_t)1 << 30;
constexpr size_t kChunkBudgetBatchedMixed = (size_t)256 << 20;

inline size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// Chunk budgets a plan may use (jk_tune.h); workspace sizes cover all.
constexpr int kChunkChoicesMb[] = {64, 128, 256, 512, 1024, 2048, 4096};

// The plan choices of the current build: the recorded ones, or those being
// timed by jk_autotune on this thread.
thread_local const jk_tuning *t_forced = nullptr;
jk_tuning plan_tuning(const jk_problem *p) { return t_forced ? *t_forced : jk::tuning_for(p); }
inline size_t tuned_budget(const jk_problem *p) { return (size_t)plan_tuning(p).chunk_mb << 20; }

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
    if (p->flags < 0 || (p->flags & ~(JK_WANT_J | JK_WANT_K | JK_B_PACKED)) != 0)
        return false;
    if (p->reserved != 0)
        return false;
    if (p->precision == JK_MIXED && p->nslice != 0 && (p->nslice < 1 || p->nslice > 5))
        return false;
    return true;
}

inline int want(const jk_problem *p)
{
    const int f = p->flags & (JK_WANT_J | JK_WANT_K);
    return f == 0 ? (JK_WANT_J | JK_WANT_K) : f;
}
inline bool packed_b(const jk_problem *p) { return (p->flags & JK_B_PACKED) != 0; }

// Slabs per chunk of the half-transform workspace.
int chunk_slabs(const jk_problem *p, size_t budget)
{
    size_t per = 2 * (size_t)p->nao * (size_t)(p->ndens * p->rank) * sizeof(double);
    i64 qc = (i64)(budget / (per ? per : 1));
    // a multiple of 16 / gcd(rank, 16) slabs, so that a full chunk's exchange
    // depth qc * rank is a whole number of 16-deep stages (no masked stage)
    i64 m = 16;
    for (i64 g = p->rank; g % 2 == 0 && m > 1; g /= 2)
        m /= 2;
    if (qc >= m)
        qc -= qc % m;
    if (qc < 1)
        qc = 1;
    if (qc > p->naux)
        qc = p->naux;
    return (int)qc;
}

struct FwdPlan {
    int qc, ldw, npb, plen, ndp, nsplit;
    int nsplit_sym;     // exchange splits when C_L = C_R (upper-triangle tiles)
    bool packed;        // B slabs stored as packed upper triangles
    i64 slab;           // doubles per slab of B
    size_t o_cc, o_d, o_s, o_part, o_g, o_x, o_y, o_kp, total;
};

FwdPlan plan_forward(const jk_problem *p, size_t budget = kChunkBudget)
{
    FwdPlan f;
    const i64 nao = p->nao, nd = p->ndens, r = p->rank, R = nd * r;
    const i64 npos = nao * nao;
    f.qc = chunk_slabs(p, budget);
    f.ldw = (int)(f.qc * r);
    f.ndp = (int)(((nd + 7) / 8) * 8);
    f.packed = packed_b(p);
    f.slab = f.packed ? jk::pk_size((int)nao) : npos;
    // gamma runs over the stored positions of a slab
    // gamma: packed slabs stream their positions in blocks of plen; full
    // squares read their upper triangles in row groups of plen rows, npb
    // pairs of groups (coulomb_upper.hpp)
    if (f.packed)
        f.npb = jk::project_nblocks(f.slab, (int)p->naux, (int)nd, &f.plen);
    else
        f.npb = jk::project_upper_blocks((int)nao, (int)p->naux, (int)((nd + 7) / 8), &f.plen);
    Carve c;
    f.o_cc = c.take(sizeof(double) * nao * 2 * R);
    f.o_d = c.take(sizeof(double) * nd * npos);
    f.o_s = c.take(f.packed ? sizeof(double) * nd * f.slab : 0);
    f.o_part = c.take(sizeof(double) * (size_t)f.npb * p->naux * f.ndp);
    f.o_g = c.take(sizeof(double) * nd * p->naux);
    f.o_x = c.take(sizeof(double) * nd * nao * (size_t)f.ldw);
    f.o_y = c.take(sizeof(double) * nd * nao * (size_t)f.ldw);
    f.nsplit = jk::exchange_nsplit((int)nao, (int)nd, f.ldw);
    f.nsplit_sym = jk::exchange_nsplit((int)nao, (int)nd, f.ldw, 1);
    const int nsmax = f.nsplit > f.nsplit_sym ? f.nsplit : f.nsplit_sym;
    f.o_kp = c.take(nsmax > 1 ? sizeof(double) * (size_t)nsmax * nd * npos : 0);
    f.total = c.off;
    return f;
}

// Slabs per chunk of the derivative: X, Y and the slab blocks [P' | R'] of one
// chunk in the budget (4 GB: fewer, larger launches, so that each
// launch's last partial round of workgroups is a smaller share of it).
constexpr size_t kChunkBudgetVjp = (size_t)4 << 30;
int chunk_slabs_vjp(const jk_problem *p)
{
    size_t per = 4 * (size_t)p->nao * (size_t)(p->ndens * p->rank) * sizeof(double);
    size_t budget = kChunkBudgetVjp;
    if (p->flags & JK_B_PACKED) {
        // the chunk's slabs unpacked to full squares, on a budget of their own
        per += (size_t)p->nao * (size_t)p->nao * sizeof(double);
        budget *= 2;
    }
    i64 qc = (i64)(budget / (per ? per : 1));
    if (qc < 1)
        qc = 1;
    if (qc > p->naux)
        qc = p->naux;
    return (int)qc;
}

struct VjpPlan {
    int qc, ldw, npb, plen, ndp, nsplit_c;
    bool paired;        // omega and gamma in one pass over B (2 nd <= 16)
    bool packed;        // JK_B_PACKED: chunks unpacked into o_bu, packed W, D, E
    size_t o_cc, o_d, o_e, o_part, o_g, o_om, o_omx, o_x, o_y, o_pr, o_dcp;
    size_t o_bu, o_wdp, o_ep, total;
};

VjpPlan plan_vjp(const jk_problem *p)
{
    VjpPlan f;
    const i64 nao = p->nao, nd = p->ndens, r = p->rank, R = nd * r, naux = p->naux;
    f.packed = packed_b(p);
    // positions per slab of B as stored (the projections stream them)
    const i64 npos = f.packed ? nao * (nao + 1) / 2 : nao * nao;
    f.qc = chunk_slabs_vjp(p);
    f.ldw = (int)(f.qc * r);
    f.ndp = (int)(((nd + 7) / 8) * 8);
    f.npb = jk::project_nblocks(npos, (int)naux, (int)nd, &f.plen);
    f.nsplit_c = jk::vjp_stage_c_nsplit((int)nao, (int)R, f.qc);
    f.paired = 2 * nd <= 16;
    size_t part = (size_t)f.npb * naux * f.ndp;
    if (f.paired) {
        // 2 nd <= 8: one group of the 8-wide projection; else the 16-wide one
        int plen2;
        const size_t p2 = 2 * nd <= 8
                              ? (size_t)jk::project_nblocks(npos, (int)naux, (int)(2 * nd), &plen2) * naux * 8
                              : (size_t)jk::project16_nblocks(npos, (int)naux, &plen2) * naux * 16;
        part = part > p2 ? part : p2;
        if (!f.packed) {
            // full squares: [W | D] folded onto the upper triangles
            int G;
            const size_t p3 = (size_t)jk::project_upper_blocks((int)nao, (int)naux, 1, &G) * naux *
                              (2 * nd <= 8 ? 8 : 16);
            part = part > p3 ? part : p3;
        }
    }
    if (!f.packed) {
        // full squares, W and D projected on their own (groups of 8)
        int G;
        const size_t p4 = (size_t)jk::project_upper_blocks((int)nao, (int)naux, (int)((nd + 7) / 8), &G) *
                          naux * f.ndp;
        part = part > p4 ? part : p4;
    }
    Carve c;
    const i64 nsq = nao * nao;
    f.o_cc = c.take(sizeof(double) * nao * 2 * R);
    // [W | D]: the cotangent copied in front of the densities (folded in
    // place for full squares; paired, the two in one pass over B)
    f.o_d = c.take(sizeof(double) * (f.paired || !f.packed ? 2 : 1) * nd * nsq);
    f.o_e = c.take(sizeof(double) * nd * nsq);
    f.o_part = c.take(sizeof(double) * part);
    f.o_g = c.take(sizeof(double) * nd * naux);
    f.o_om = c.take(sizeof(double) * (f.paired ? 2 : 1) * nd * naux);   // paired: [omega | gamma]
    f.o_omx = c.take(sizeof(double) * naux * R);
    f.o_x = c.take(sizeof(double) * nd * nao * (size_t)f.ldw);
    f.o_y = c.take(sizeof(double) * nd * nao * (size_t)f.ldw);
    f.o_pr = c.take(sizeof(double) * (size_t)f.qc * nao * 2 * R);
    f.o_dcp = c.take(sizeof(double) * (size_t)f.nsplit_c * nao * 2 * R);
    if (f.packed) {
        // the chunk's slabs as full squares (stage C, their last reader, runs
        // on the stream that unpacks the next chunk); W, D and E as packed
        // sums over each symmetric pair of positions
        f.o_bu = c.take(sizeof(double) * (size_t)f.qc * nsq);
        f.o_wdp = c.take(sizeof(double) * 2 * nd * npos);
        f.o_ep = c.take(sizeof(double) * nd * npos);
    } else {
        f.o_bu = f.o_wdp = f.o_ep = 0;
    }
    f.total = c.off;
    return f;
}

#define JK_TRY(expr)                                                                               \
    do {                                                                                           \
        hipError_t _e = (expr);                                                                    \
        if (_e != hipSuccess)                                                                      \
            return JK_EHIP;                                                                        \
    } while (0)

// Mixed-precision plan: the FP64 plan (gamma, J, chunk buffers) plus int8
// digit planes of [C_L | C_R] and, double-buffered so that consecutive
// chunks overlap, the digit planes of B, the half-transformed factors XY and
// their digit planes.
struct MixPlan {
    FwdPlan f;
    int ns, mp, kp, cp, jp, nsplit;
    int mpb;                  // rows per slab of B's planes (X/Y planes: mp)
    int cp_sym, nsplit_sym;   // X-only columns and triangle splits (C_L = C_R)
    size_t bp_bytes, xy_bytes, xyp_bytes;
    size_t o_bp[2], o_eb[2], o_xy[2], o_xyp[2], o_exy[2], o_cp, o_ec, o_kp, total;
    size_t o_pm[2];           // the half-transform's row maxima per tile (single builds)
};

inline i64 pad_to(i64 x, i64 m) { return ((x + m - 1) / m) * m; }

MixPlan plan_mixed(const jk_problem *p, size_t budget = kChunkBudget)
{
    MixPlan x;
    x.f = plan_forward(p, budget);
    const i64 nao = p->nao, nd = p->ndens, r = p->rank, R = nd * r;
    x.ns = jk::mixed_nslice();
    x.mp = (int)pad_to(nao, jk::mixed_row_pad());
    x.mpb = (int)pad_to(nao, jk::mixed_b_row_pad());
    x.kp = (int)pad_to(nao, jk::mixed_k_pad());
    x.cp = (int)pad_to(2 * R, jk::mixed_row_pad());
    x.jp = (int)pad_to((i64)x.f.qc * r, jk::mixed_k_pad());
    x.nsplit = jk::ex_mixed_nsplit(x.mp, (int)nd, x.jp / jk::mixed_k_block());
    x.cp_sym = (int)pad_to(R, jk::mixed_row_pad());
    x.nsplit_sym = jk::ex_mixed_nsplit(x.mp, (int)nd, x.jp / jk::mixed_k_block(), 1);
    const int nsmax = x.nsplit > x.nsplit_sym ? x.nsplit : x.nsplit_sym;
    x.bp_bytes = (size_t)x.ns * x.f.qc * x.mpb * x.kp;
    x.xy_bytes = sizeof(double) * (size_t)x.f.qc * nao * 2 * R;
    x.xyp_bytes = (size_t)x.ns * 2 * nd * x.mp * x.jp;
    Carve c;
    c.off = x.f.total;
    // XY buffer 0 is the FP64 path's X and Y chunk buffers, carved back to
    // back (together at least qc * nao * 2R doubles).
    x.o_xy[0] = x.f.o_x;
    x.o_xy[1] = c.take(x.xy_bytes);
    for (int b = 0; b < 2; b++) {
        x.o_bp[b] = c.take(x.bp_bytes);
        x.o_eb[b] = c.take(sizeof(int) * (size_t)x.f.qc * x.mpb);
        x.o_xyp[b] = c.take(x.xyp_bytes);
        x.o_exy[b] = c.take(sizeof(int) * (size_t)2 * nd * x.mp);
    }
    x.o_cp = c.take((size_t)x.ns * x.cp * x.kp);
    x.o_ec = c.take(sizeof(int) * (size_t)x.cp);
    x.o_kp = c.take(sizeof(double) * (size_t)nsmax * nd * nao * nao);
    // sized for both sides (the X-only case has fewer column tiles and keys)
    const size_t pm = jk::xy_rowmax_pm_doubles(x.f.qc, x.mpb, x.cp, (int)r, (int)(2 * nd));
    for (int b = 0; b < 2; b++)
        x.o_pm[b] = c.take(sizeof(double) * pm);
    x.total = c.off;
    return x;
}

// Second stream per device for the HBM-bound slicing work of the mixed
// build (default priority, non-blocking, kept for the life of the process).
hipError_t aux_stream(hipStream_t *out)
{
    static std::mutex mu;
    static std::map<int, hipStream_t> streams;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    std::lock_guard<std::mutex> lk(mu);
    auto it = streams.find(dev);
    if (it == streams.end()) {
        hipStream_t st = nullptr;
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e != hipSuccess)
            return e;
        it = streams.emplace(dev, st).first;
    }
    *out = it->second;
    return hipSuccess;
}

// Events of one call (destroyed when the call returns; a pending event is
// released by the runtime once it completes).
struct EventSet {
    hipEvent_t ev[9] = {};
    int n = 0;
    hipError_t create(int count)
    {
        for (n = 0; n < count; n++) {
            hipError_t e = hipEventCreateWithFlags(&ev[n], hipEventDisableTiming);
            if (e != hipSuccess)
                return e;
        }
        return hipSuccess;
    }
    ~EventSet()
    {
        for (int i = 0; i < n; i++)
            (void)hipEventDestroy(ev[i]);
    }
};

// One stream of Cholesky vectors feeding the exchange sum:
//     K += scale * sum_{Q < naux} B^Q D B^Q.
// The plain build has one segment (B, scale 1); the Fock combination adds a
// segment per exchange operator (e.g. the long-range factor set).
struct KSeg {
    const double *B;
    int naux;
    double scale;
};

// What a build writes: J and K (the plain build, as selected by flags), or
// one combined F = cj J + sum over segments of scale K (when F is set).
struct BuildOut {
    double *J = nullptr, *K = nullptr;
    double *F = nullptr;
    double cj = 0.0;
};

// The Coulomb part: gamma_kQ = <D_k, B^Q> in FP64, then
// out (+)= scale sum_Q gamma_kQ B^Q.  Packed slabs: gamma pairs B^Q with the
// packed S_k = D_k + D_k^T (diagonal once), J runs over the packed positions
// into the D buffer and is written out in full by the unpack pass.
jk_status coulomb_part(const FwdPlan &f, int nao, int naux, int nd, int r, const double *B,
                       const double *CL, const double *CR, double *out, double scale,
                       int accumulate, char *ws, hipStream_t s)
{
    double *D = (double *)(ws + f.o_d);
    double *part = (double *)(ws + f.o_part);
    double *g = (double *)(ws + f.o_g);
    JK_TRY(jk::launch_density(CL, CR, D, nao, nd, r, s));
    if (!f.packed) {
        // the upper triangles of the symmetric slabs: D folded onto its own
        JK_TRY(jk::launch_fold_upper(D, nao, nd, s));
        JK_TRY(jk::launch_project_upper(B, D, part, g, nao, naux, nd, s));
        JK_TRY(jk::launch_coulomb_upper(B, g, out, nao, naux, nd, s, scale, accumulate));
        return JK_OK;
    }
    double *S = (double *)(ws + f.o_s);
    JK_TRY(jk::launch_sym_pack(D, S, nao, nd, s));
    JK_TRY(jk::launch_project(B, S, part, g, naux, nd, f.slab, s));
    JK_TRY(jk::launch_coulomb(B, g, D, naux, nd, f.slab, s));
    JK_TRY(jk::launch_unpack_sym(D, out, nao, nd, scale, accumulate, s));
    return JK_OK;
}

jk_status build_fp64(const jk_problem *p, const double *B, const KSeg *seg, int nseg,
                     const double *CL, const double *CR, const BuildOut &o, char *ws,
                     hipStream_t s)
{
    const jk_tuning tu = plan_tuning(p);
    const FwdPlan f = plan_forward(p, (size_t)tu.chunk_mb << 20);
    const int nao = (int)p->nao, naux = (int)p->naux, nd = (int)p->ndens, r = (int)p->rank;
    const i64 npos = (i64)nao * nao;
    const int w = want(p);
    const bool fused = o.F != nullptr;
    double *Kout = fused ? o.F : o.K;
    double *Cc = (double *)(ws + f.o_cc);
    double *Xw = (double *)(ws + f.o_x);
    double *Yw = (double *)(ws + f.o_y);

    if (!fused && (w & JK_WANT_J)) {
        jk_status st = coulomb_part(f, nao, naux, nd, r, B, CL, CR, o.J, 1.0, 0, ws, s);
        if (st != JK_OK)
            return st;
    }
    const bool want_k = fused ? nseg > 0 : (w & JK_WANT_K) != 0;
    if (want_k) {
        // K accumulates over the Q-chunks of every segment in nsplit partial
        // buffers (or in the output itself when nsplit == 1), summed in fixed
        // order at the end.  The same factor for both sides (C_L = C_R,
        // symmetric densities): only X is formed, K = sum X X^T on the
        // upper-triangle tiles, and the lower triangle is mirrored at the end.
        const bool sym = CL == CR;
        const int ns = sym ? f.nsplit_sym : f.nsplit;
        double *Kp = ns > 1 ? (double *)(ws + f.o_kp) : Kout;
        double *Yx = sym ? Xw : Yw;
        JK_TRY(jk::launch_pack_c(CL, CR, Cc, nao, nd, r, s));
        bool first = true;
        for (int sgi = 0; sgi < nseg; sgi++) {
            const KSeg &sg = seg[sgi];
            for (int q0 = 0; q0 < sg.naux; q0 += f.qc) {
                int nq = (sg.naux - q0) < f.qc ? (sg.naux - q0) : f.qc;
                JK_TRY(jk::launch_half_transform(sg.B, Cc, Xw, Yw, nao, nd, r, q0, nq, f.ldw, s,
                                                 sym ? nd * r : 2 * nd * r, f.packed ? 1 : 0,
                                                 tu.ht_tile));
                JK_TRY(jk::launch_exchange(Xw, Yx, Kp, nao, nd, nq * r, f.ldw, ns, !first, s, sym,
                                           sg.scale));
                first = false;
            }
        }
        if (ns > 1)
            JK_TRY(jk::launch_sum_splits(Kp, Kout, (i64)nd * npos, ns, s));
        if (sym)
            JK_TRY(jk::launch_mirror_upper(Kout, nao, nd, s));
    }
    if (fused && (o.cj != 0.0 || !want_k)) {
        // F (+)= cj J (J is symmetric, so the order against the mirror does
        // not matter); with no exchange term this writes F = cj J.
        jk_status st = coulomb_part(f, nao, naux, nd, r, B, CL, CR, o.F, o.cj, want_k ? 1 : 0, ws,
                                    s);
        if (st != JK_OK)
            return st;
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
    // Packed B: the projections and the affine term run over the packed
    // positions, with W, D and E folded onto them (each symmetric pair of
    // positions summed: <W, B^Q> over the square is the packed dot product);
    // every chunk is unpacked to full squares for the half-transform and
    // stage C, and stage D writes the packed gradient.
    const bool pk = f.packed;
    const i64 npk = pk ? (i64)nao * (nao + 1) / 2 : npos;
    double *WDp = pk ? (double *)(ws + f.o_wdp) : nullptr;
    double *Ep = pk ? (double *)(ws + f.o_ep) : nullptr;
    const int has_w = W != nullptr, has_v = V != nullptr;
    const bool want_db = dB != nullptr, want_dc = dCL != nullptr;
    double *Cc = (double *)(ws + f.o_cc);
    double *D = (double *)(ws + f.o_d);
    double *E = (double *)(ws + f.o_e);
    double *part = (double *)(ws + f.o_part);
    double *g = (double *)(ws + f.o_g);
    double *om = (double *)(ws + f.o_om);
    double *omx = (double *)(ws + f.o_omx);
    double *Xw = (double *)(ws + f.o_x);
    double *Yw = (double *)(ws + f.o_y);
    double *L = (double *)(ws + f.o_pr);
    double *dCp = (double *)(ws + f.o_dcp);
    // The same factor for both sides (C_L = C_R, symmetric densities): Y = X,
    // so the half-transforms form X only and both stage-B products read it.
    const bool sym = CL == CR;
    double *Yx = sym ? Xw : Yw;

    JK_TRY(jk::launch_pack_c(CL, CR, Cc, nao, nd, r, s));
    if (has_w && want_db && f.paired) {
        // omega_kQ = <W_k, B^Q> and gamma_kQ = <D_k, B^Q> in one pass over B:
        // the 2 nd matrices [W | D] against each slab; E = D - 2 D^T.
        double *WD = D;
        D = WD + (i64)nd * npos;
        g = om + (i64)nd * naux;
        JK_TRY(hipMemcpyAsync(WD, W, sizeof(double) * (size_t)nd * npos, hipMemcpyDeviceToDevice, s));
        JK_TRY(jk::launch_density(CL, CR, D, nao, nd, r, s));
        JK_TRY(jk::launch_vjp_e_matrix(D, E, nao, nd, s));
        if (pk) {
            JK_TRY(jk::launch_sym_pack(WD, WDp, nao, 2 * nd, s));
            if (2 * nd <= 8)
                JK_TRY(jk::launch_project(B, WDp, part, om, naux, 2 * nd, npk, s));
            else
                JK_TRY(jk::launch_project16(B, WDp, part, om, naux, 2 * nd, npk, s));
        } else {
            // the upper triangles of the symmetric slabs: [W | D] folded onto
            // their own (E is formed from D above, before the fold)
            JK_TRY(jk::launch_fold_upper(WD, nao, 2 * nd, s));
            JK_TRY(jk::launch_project_upper(B, WD, part, om, nao, naux, 2 * nd, s, 2 * nd > 8));
        }
        JK_TRY(jk::launch_omega_expand(om, omx, naux, nd, r, s));
    } else if (has_w && pk) {
        // omega_kQ = <W_k, B^Q>; for dB also gamma_kQ = <D_k, B^Q> and E = D - 2 D^T.
        JK_TRY(jk::launch_sym_pack(W, WDp, nao, nd, s));
        JK_TRY(jk::launch_project(B, WDp, part, om, naux, nd, npk, s));
        JK_TRY(jk::launch_omega_expand(om, omx, naux, nd, r, s));
        if (want_db) {
            JK_TRY(jk::launch_density(CL, CR, D, nao, nd, r, s));
            JK_TRY(jk::launch_sym_pack(D, WDp + (i64)nd * npk, nao, nd, s));
            JK_TRY(jk::launch_project(B, WDp + (i64)nd * npk, part, g, naux, nd, npk, s));
            JK_TRY(jk::launch_vjp_e_matrix(D, E, nao, nd, s));
        }
    } else if (has_w) {
        // The same from a folded copy of W (then D), in the row groups of the
        // paired pass: omega comes out bit for bit as there.
        double *Wc = D;
        D = Wc + (i64)nd * npos;
        JK_TRY(hipMemcpyAsync(Wc, W, sizeof(double) * (size_t)nd * npos, hipMemcpyDeviceToDevice, s));
        JK_TRY(jk::launch_fold_upper(Wc, nao, nd, s));
        JK_TRY(jk::launch_project_upper(B, Wc, part, om, nao, naux, nd, s));
        JK_TRY(jk::launch_omega_expand(om, omx, naux, nd, r, s));
        if (want_db) {
            JK_TRY(jk::launch_density(CL, CR, D, nao, nd, r, s));
            JK_TRY(jk::launch_vjp_e_matrix(D, E, nao, nd, s));
            JK_TRY(jk::launch_fold_upper(D, nao, nd, s));
            JK_TRY(jk::launch_project_upper(B, D, part, g, nao, naux, nd, s));
        }
    }
    // the affine term's matrices as the positions of dB are stored
    const double *Wa = W, *Ea = E;
    if (pk && has_w && want_db) {
        JK_TRY(jk::launch_sym_pack(E, Ep, nao, nd, s));
        Wa = WDp;                                 // [W | D] packed, W first
        Ea = Ep;
    }
    // Stage B's two products run side by side on two streams:
    //   main: HT(c), B[P'](c), C(c), D(c), affine(c)
    //   aux:  B[R'](c)
    // aux's B[R'](c) waits for HT(c) (it reads X), whose event main records
    // after every reader of chunk c - 1's slab blocks; main waits for B[R'](c)
    // before stage C.  Stage C beside stage D (on the second stream) took 2%
    // longer than the two in sequence.
    hipStream_t a = nullptr;
    JK_TRY(aux_stream(&a));
    EventSet ev;
    JK_TRY(ev.create(2));
    hipEvent_t ev_x = ev.ev[0], ev_br = ev.ev[1];
    const int tile = plan_tuning(p).ht_tile;
    for (int q0 = 0; q0 < naux; q0 += f.qc) {
        const int nq = (naux - q0) < f.qc ? (naux - q0) : f.qc;
        // the slabs the half-transform and stage C read: B itself, or this
        // chunk unpacked
        const double *Bs = B;
        int qs = q0;
        if (pk && (has_v || want_dc)) {
            double *Bu = (double *)(ws + f.o_bu);
            JK_TRY(jk::launch_unpack_slabs(B, Bu, nao, q0, nq, s));
            Bs = Bu;
            qs = 0;
        }
        if (has_v)
            JK_TRY(jk::launch_half_transform(Bs, Cc, Xw, Yw, nao, nd, r, qs, nq, f.ldw, s,
                                             sym ? R : 2 * R, 0, tile, "vjp_half_transform"));
        JK_TRY(hipEventRecord(ev_x, s));         // X, Y of this chunk; D of the last done
        JK_TRY(hipStreamWaitEvent(a, ev_x, 0));
        JK_TRY(jk::launch_vjp_stage_b_one(1, V, Xw, Cc, omx, L, nao, nd, r, q0, nq * r, f.ldw, has_v,
                                          has_w, a));
        JK_TRY(hipEventRecord(ev_br, a));
        JK_TRY(jk::launch_vjp_stage_b_one(0, V, Yx, Cc, omx, L, nao, nd, r, q0, nq * r, f.ldw, has_v,
                                          has_w, s));
        JK_TRY(hipStreamWaitEvent(s, ev_br, 0));
        if (want_dc)
            JK_TRY(jk::launch_vjp_stage_c(Bs, L, dCp, nao, R, qs, nq, f.nsplit_c, q0 > 0, s));
        if (want_db) {
            if (pk)
                JK_TRY(jk::launch_vjp_stage_d_packed(L, Cc, dB, nao, R, q0, nq, s));
            else
                JK_TRY(jk::launch_vjp_stage_d(L, Cc, dB, nao, R, q0, nq, s));
            if (has_w)
                JK_TRY(jk::launch_vjp_db_affine(g, om, Wa, Ea, dB, nd, naux, npk, q0, nq, s));
        }
    }
    if (want_dc)
        JK_TRY(jk::launch_vjp_dc_finish(dCp, dCL, dCR, nao, nd, r, f.nsplit_c, s));
    return JK_OK;
}

// Digit planes of a whole B made once by jk_slice_b (jk.h): row exponents of
// the naux * mp plane rows, then the planes, K-blocked over all slabs.
struct SliceLayout {
    int mp, kp;
    size_t o_exp, o_planes, total;
    i64 kbstride, pstride;
};

SliceLayout slice_layout(const jk_problem *p)
{
    SliceLayout L;
    L.mp = (int)pad_to(p->nao, jk::mixed_b_row_pad());
    L.kp = (int)pad_to(p->nao, jk::mixed_k_pad());
    const int KB = jk::mixed_k_block();
    L.kbstride = (i64)p->naux * L.mp * KB;
    L.pstride = L.kbstride * (L.kp / KB);
    Carve c;
    L.o_exp = c.take(sizeof(int) * (size_t)p->naux * L.mp);
    L.o_planes = c.take((size_t)jk::mixed_nslice() * L.pstride);
    L.total = c.off;
    return L;
}

jk_status build_mixed(const jk_problem *p, const double *B, const KSeg *seg, int nseg,
                      const double *CL, const double *CR, const BuildOut &o, char *ws,
                      hipStream_t s, const char *pre = nullptr)
{
    const MixPlan x = plan_mixed(p, tuned_budget(p));
    const FwdPlan &f = x.f;
    const int nao = (int)p->nao, naux = (int)p->naux, nd = (int)p->ndens, r = (int)p->rank;
    const int R = nd * r, R2 = 2 * R;
    if (!jk::mixed_rowmax_ok(R2) || (p->nslice != 0 && p->nslice != jk::mixed_nslice()))
        return JK_EUNSUPPORTED;
    if (f.packed && !jk::mixed_packed_ok(nao, x.kp))
        return JK_EUNSUPPORTED;
    const i64 npos = (i64)nao * nao;
    const int w = want(p);
    const bool fused = o.F != nullptr;
    double *K = fused ? o.F : o.K;
    // gamma and J stay FP64 (the same kernels as the FP64 path).
    if (!fused && (w & JK_WANT_J)) {
        jk_status st = coulomb_part(f, nao, naux, nd, r, B, CL, CR, o.J, 1.0, 0, ws, s);
        if (st != JK_OK)
            return st;
    }
    const bool want_k = fused ? nseg > 0 : (w & JK_WANT_K) != 0;
    auto fock_j = [&]() -> jk_status {
        if (fused && (o.cj != 0.0 || !want_k))
            return coulomb_part(f, nao, naux, nd, r, B, CL, CR, o.F, o.cj, want_k ? 1 : 0, ws, s);
        return JK_OK;
    };
    if (!want_k)
        return fock_j();
    // The Q-chunks of every segment, in order: slab pointer, slab count,
    // exchange scale.
    struct Chunk {
        const double *B;
        int q0, nq;
        double scale;
    };
    std::vector<Chunk> chunks;
    for (int sgi = 0; sgi < nseg; sgi++)
        for (int q0 = 0; q0 < seg[sgi].naux; q0 += f.qc)
            chunks.push_back({seg[sgi].B + (i64)q0 * f.slab, q0,
                              (seg[sgi].naux - q0) < f.qc ? (seg[sgi].naux - q0) : f.qc,
                              seg[sgi].scale});
    // B's digit planes: made here chunk by chunk, or read from the caller's
    // prepared planes of the whole B (one segment only)
    if (pre && nseg != 1)
        return JK_EINVAL;
    const SliceLayout SL = slice_layout(p);
    double *Cc = (double *)(ws + f.o_cc);
    int8_t *Cp = (int8_t *)(ws + x.o_cp);
    int *eC = (int *)(ws + x.o_ec);
    // The same factor for both sides (C_L = C_R): X only, K on the upper
    // triangle, mirrored at the end.
    const bool sym = CL == CR;
    const int nsplit = sym ? x.nsplit_sym : x.nsplit;
    const int ncol = sym ? R : R2, nkey = sym ? nd : 2 * nd, cpx = sym ? x.cp_sym : x.cp;
    double *Kp = nsplit > 1 ? (double *)(ws + x.o_kp) : K;
    const int KB = jk::mixed_k_block();
    // K-blocked plane strides (slice_core.hpp): kbstride = rows * 32 bytes
    const i64 bkb = pre ? SL.kbstride : (i64)f.qc * x.mpb * KB;
    const i64 bps = pre ? SL.pstride : bkb * (x.kp / KB);
    const i64 ckb = (i64)x.cp * KB, cps = ckb * (x.kp / KB);
    const i64 xkb = (i64)2 * nd * x.mp * KB, xps = xkb * (x.jp / KB);
    const int nchunk = (int)chunks.size();
    auto nq_of = [&](int c) { return chunks[c].nq; };
    auto nkb_of = [&](int c) { return (int)(pad_to((i64)nq_of(c) * r, jk::mixed_k_pad()) / KB); };
    auto Bp = [&](int c) {
        return pre ? (int8_t *)(pre + SL.o_planes) + (i64)chunks[c].q0 * x.mpb * KB
                   : (int8_t *)(ws + x.o_bp[c & 1]);
    };
    auto eB = [&](int c) {
        return pre ? (int *)(pre + SL.o_exp) + (i64)chunks[c].q0 * x.mpb : (int *)(ws + x.o_eb[c & 1]);
    };
    auto XY = [&](int c) { return (double *)(ws + x.o_xy[c & 1]); };
    auto XYp = [&](int c) { return (int8_t *)(ws + x.o_xyp[c & 1]); };
    auto eXY = [&](int c) { return (int *)(ws + x.o_exy[c & 1]); };
    auto PM = [&](int c) { return (double *)(ws + x.o_pm[c & 1]); };

    // Two streams.  Main stream s: the MFMA-bound products, ht(c + 1) then
    // ex(c).  Auxiliary stream a: the HBM-bound slicing, slice_b(c + 2), then
    // rowmax / slice_xy(c + 1).  Buffers are double-buffered by chunk parity;
    // every reuse waits for the last reader of the previous occupant:
    //   Bp/eB[c]   written by slice_b(c),  read by ht(c)
    //   XY/PM[c]   written by ht(c),       read by rowmax/slice_xy(c)
    //   XYp/eXY[c] written by slice_xy(c), read by ex(c)
    hipStream_t a = nullptr;
    JK_TRY(aux_stream(&a));
    EventSet E;
    JK_TRY(E.create(9));
    hipEvent_t fork = E.ev[0], sb[2] = {E.ev[1], E.ev[2]}, ht[2] = {E.ev[3], E.ev[4]},
               sx[2] = {E.ev[5], E.ev[6]}, ex[2] = {E.ev[7], E.ev[8]};
    auto slice_b = [&](int c) -> jk_status {
        if (pre) {              // prepared planes: nothing to make
            JK_TRY(hipEventRecord(sb[c & 1], a));
            return JK_OK;
        }
        if (f.packed)
            JK_TRY(jk::launch_slice_b_packed(chunks[c].B, f.slab, nq_of(c), nao, x.mpb, x.kp / KB,
                                             Bp(c), bps, bkb, eB(c), a));
        else
            JK_TRY(jk::launch_slice_b(chunks[c].B, npos, nao, nq_of(c), nao, nao, x.mpb,
                                      x.kp / KB, Bp(c), bps, bkb, eB(c), a));
        JK_TRY(hipEventRecord(sb[c & 1], a));
        return JK_OK;
    };
    auto slice_xy = [&](int c) -> jk_status {
        JK_TRY(jk::launch_xy_rowmax_pm(PM(c), nao, nq_of(c), nkey, r, x.mpb, x.mp, cpx, eXY(c), a));
        JK_TRY(jk::launch_slice_xy(XY(c), nao, nkey, r, x.mp, nq_of(c) * r, nkb_of(c), XYp(c), xps, xkb,
                                   eXY(c), a));
        JK_TRY(hipEventRecord(sx[c & 1], a));
        return JK_OK;
    };
    auto half = [&](int c) -> jk_status {
        JK_TRY(hipStreamWaitEvent(s, sb[c & 1], 0));
        if (c >= 2)
            JK_TRY(hipStreamWaitEvent(s, sx[c & 1], 0));    // XY[c] free
        JK_TRY(jk::launch_ht_mixed(Bp(c), bps, bkb, eB(c), Cp, cps, ckb, eC, XY(c), nao, ncol, nq_of(c),
                                   x.mpb, cpx, x.kp / KB, s, PM(c), r));
        JK_TRY(hipEventRecord(ht[c & 1], s));
        return JK_OK;
    };
    auto exch = [&](int c) -> jk_status {
        JK_TRY(hipStreamWaitEvent(s, sx[c & 1], 0));
        const int8_t *Xp = XYp(c), *Yp = sym ? Xp : XYp(c) + (i64)nd * x.mp * KB;
        const int *eX = eXY(c), *eY = sym ? eX : eXY(c) + (size_t)nd * x.mp;
        JK_TRY(jk::launch_ex_mixed(Xp, Yp, xps, xkb, eX, eY, Kp, nao, nd, x.mp, nkb_of(c), nsplit, c > 0, s,
                                   sym, chunks[c].scale));
        JK_TRY(hipEventRecord(ex[c & 1], s));
        return JK_OK;
    };
#define JK_STEP(expr)                                                                              \
    do {                                                                                           \
        jk_status st_ = (expr);                                                                    \
        if (st_ != JK_OK)                                                                          \
            return st_;                                                                            \
    } while (0)

    JK_TRY(jk::launch_pack_c(CL, CR, Cc, nao, nd, r, s));
    // digits of [C_L | C_R]: row c, inner n, element Cc[n][c]
    JK_TRY(jk::launch_slice_rows(Cc, 0, 1, R2, 1, R2, nao, x.cp, x.kp / KB, Cp, cps, ckb, eC, s));
    JK_TRY(hipEventRecord(fork, s));
    JK_TRY(hipStreamWaitEvent(a, fork, 0));
    JK_STEP(slice_b(0));
    if (nchunk > 1)
        JK_STEP(slice_b(1));
    JK_STEP(half(0));
    JK_TRY(hipStreamWaitEvent(a, ht[0], 0));
    JK_STEP(slice_xy(0));
    for (int c = 0; c < nchunk; c++) {
        if (c + 1 < nchunk)
            JK_STEP(half(c + 1));
        JK_STEP(exch(c));
        if (c + 2 < nchunk) {
            JK_TRY(hipStreamWaitEvent(a, ht[c & 1], 0));     // Bp[c] free
            JK_STEP(slice_b(c + 2));
        }
        if (c + 1 < nchunk) {
            JK_TRY(hipStreamWaitEvent(a, ht[(c + 1) & 1], 0));
            if (c >= 1)
                JK_TRY(hipStreamWaitEvent(a, ex[(c + 1) & 1], 0));   // XYp[c+1] free
            JK_STEP(slice_xy(c + 1));
        }
    }
#undef JK_STEP
    if (nsplit > 1)
        JK_TRY(jk::launch_sum_splits(Kp, K, (i64)nd * npos, nsplit, s));
    if (sym)
        JK_TRY(jk::launch_mirror_upper(K, nao, nd, s));
    return fock_j();
}

// Two events with timing enabled (for jk_autotune), destroyed on return.
struct TimedEvents {
    hipEvent_t ev[2] = {};
    int n = 0;
    hipError_t create()
    {
        for (n = 0; n < 2; n++) {
            hipError_t e = hipEventCreate(&ev[n]);
            if (e != hipSuccess)
                return e;
        }
        return hipSuccess;
    }
    ~TimedEvents()
    {
        for (int i = 0; i < n; i++)
            (void)hipEventDestroy(ev[i]);
    }
};

// Largest forward (or mixed) plan over the chunk budgets a plan may use.
size_t forward_bytes(const jk_problem *p)
{
    size_t a = 0;
    for (int mb : kChunkChoicesMb) {
        const size_t b = (size_t)mb << 20;
        a = std::max(a, p->precision == JK_MIXED ? plan_mixed(p, b).total : plan_forward(p, b).total);
    }
    return a;
}

// The plain build: J and K of B as selected by flags.
jk_status build_plain(const jk_problem *p, const double *B, const double *CL, const double *CR,
                      double *J, double *K, char *ws, hipStream_t s)
{
    const KSeg seg{B, (int)p->naux, 1.0};
    BuildOut o;
    o.J = J;
    o.K = K;
    return p->precision == JK_MIXED ? build_mixed(p, B, &seg, 1, CL, CR, o, ws, s)
                                     : build_fp64(p, B, &seg, 1, CL, CR, o, ws, s);
}

// ------------------------------------------------------------------ batched
// Schedule of a batched build: the launches (phase, chunk step, tiles, table
// offset, argument) and the host image of the workspace header (member
// descriptors, then the member tables of every launch).  Each phase of the
// build is one launch over the members that take part in it.
struct BLaunch {
    int phase, step, ntiles, arg;
    size_t tab_off;     // byte offset of the launch's table in the workspace
};

struct BSchedule {
    std::vector<jk::BMember> mem;
    std::vector<size_t> region;      // workspace offset of each member's plan
    std::vector<BLaunch> launches;
    std::vector<int> tabs;           // all tables, concatenated
    size_t header_bytes = 0, total_bytes = 0;
    std::string key;                 // shape signature
};

// The plan of one batched member: the single-build plan for its class's
// chunk budget capped at 256 MB (members own their chunk buffers).
struct BPlan {
    FwdPlan f;
    MixPlan x;           // JK_MIXED members
    int tile = 0;        // FP64 half-transform: 0, 1 (4x4x4) or 4 (16x16x4, stacked slabs)
    int sym = 0;         // symmetric densities routed to the X-only path
    int nsplit = 1;      // exchange splits of the path taken
    size_t total = 0;
};

size_t batched_budget(const jk_problem *p)
{
    return std::min(p->precision == JK_MIXED ? kChunkBudgetBatchedMixed : kChunkBudgetBatched,
                    tuned_budget(p));
}

BPlan batched_plan(const jk_problem *p, bool sym_in)
{
    BPlan b;
    const size_t budget = batched_budget(p);
    if (p->precision == JK_MIXED) {
        b.x = plan_mixed(p, budget);
        b.f = b.x.f;
        b.sym = sym_in ? 1 : 0;
        b.nsplit = b.sym ? b.x.nsplit_sym : b.x.nsplit;
        b.total = b.x.total;
        return b;
    }
    b.f = plan_forward(p, budget);
    // tiles 3 and 4 run as the 16x16x4 tile over stacked slabs when the
    // chunk's slabs stay within a buffer resource's reach; 2 runs as 0.
    // Packed slabs always take the 16x16x4 engine's per-slab tile.
    const int t = plan_tuning(p).ht_tile;
    const bool fits = jk::buf_extent_ok((i64)b.f.qc * p->nao * p->nao);
    b.tile = b.f.packed ? 4 : t == 1 ? 1 : (t >= 3 && fits) ? 4 : 0;
    b.sym = (sym_in && b.tile == 4) ? 1 : 0;     // the X-only path needs the 16x16x4 tile
    b.nsplit = b.sym ? b.f.nsplit_sym : b.f.nsplit;
    b.total = b.f.total;
    return b;
}

// Register blocks of the mixed B slicer for rows of kp inner bytes (0 if
// rows are longer than the one-pass slicer takes).
int slicer_blocks(int kp)
{
    const int nj = (kp / jk::mixed_k_block() + 7) / 8;
    return nj <= 1 ? 1 : nj <= 2 ? 2 : nj <= 4 ? 4 : nj <= 8 ? 8 : 0;
}

bool batched_mixed_ok(int32_t nprob, const jk_problem *p)
{
    for (int g = 0; g < nprob; g++) {
        const MixPlan x = plan_mixed(&p[g], batched_budget(&p[g]));
        if (slicer_blocks(x.kp) == 0 || !jk::mixed_rowmax_ok(2 * (int)(p[g].ndens * p[g].rank)))
            return false;
        if (packed_b(&p[g]) && !jk::mixed_packed_ok((int)p[g].nao, x.kp))
            return false;
    }
    return true;
}

// Per-member cost of one tile of a phase (larger first in the tables).
double tile_cost(int phase, const BPlan &b, const jk_problem &p)
{
    switch (phase) {
    case jk::kPhaseProject: return (double)b.f.plen * (b.f.packed ? 1 : p.nao);
    case jk::kPhaseReduce: return (double)b.f.npb;
    case jk::kPhaseCoulomb: return (double)p.naux;
    case jk::kPhaseHalf:
    case jk::kPhaseHalf64:
    case jk::kPhaseHalf16:
    case jk::kPhaseMHalf: return (double)p.nao;
    case jk::kPhaseExchange:
    case jk::kPhaseMExchange: return (double)b.f.qc * p.rank / b.nsplit;
    default: return (double)p.nao;
    }
}

// sym: one flag per member (C_L and C_R one buffer), or empty for the
// workspace size (which does not depend on it).
BSchedule make_schedule(int32_t nprob, const jk_problem *p, const std::vector<char> &sym)
{
    BSchedule S;
    const int G = nprob;
    const bool mixed = p[0].precision == JK_MIXED;
    std::vector<BPlan> plans(G);
    int maxsteps = 0;
    for (int g = 0; g < G; g++) {
        plans[g] = batched_plan(&p[g], !sym.empty() && sym[g]);
        const int st = (int)((p[g].naux + plans[g].f.qc - 1) / plans[g].f.qc);
        maxsteps = std::max(maxsteps, st);
    }
    const int w = want(&p[0]);
    struct Pending {
        int phase, step, arg;
        std::vector<int> members;
        std::vector<int> tiles;
    };
    std::vector<Pending> pend;
    auto add = [&](int phase, int step, auto tiles_of, auto takes_part, int arg = 0) {
        Pending L{phase, step, arg, {}, {}};
        for (int g = 0; g < G; g++)
            if (takes_part(g)) {
                L.members.push_back(g);
                L.tiles.push_back(tiles_of(g));
            }
        // larger tiles first
        std::vector<int> idx(L.members.size());
        for (size_t i = 0; i < idx.size(); i++)
            idx[i] = (int)i;
        std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
            return tile_cost(phase, plans[L.members[a]], p[L.members[a]]) >
                   tile_cost(phase, plans[L.members[b]], p[L.members[b]]);
        });
        Pending O{phase, step, arg, {}, {}};
        for (int i : idx) {
            O.members.push_back(L.members[i]);
            O.tiles.push_back(L.tiles[i]);
        }
        if (!O.members.empty())
            pend.push_back(O);
    };
    auto all = [](int) { return true; };
    const bool packed = packed_b(&p[0]);
    auto rows = [&](int g) { return (int)(p[g].ndens * p[g].nao); };
    if (w & JK_WANT_J) {
        add(jk::kPhaseDensity, 0, [&](int g) { return jk::density_tiles((int)p[g].nao, (int)p[g].ndens); }, all);
        add(packed ? jk::kPhaseSymPack : jk::kPhaseFoldUpper, 0, rows, all);
        add(jk::kPhaseProject, 0,
            [&](int g) { return jk::project_tiles((int)p[g].naux, (int)p[g].ndens, plans[g].f.npb); }, all);
        add(jk::kPhaseReduce, 0, [&](int g) { return jk::reduce_tiles((int)p[g].naux, (int)p[g].ndens); },
            all);
        add(jk::kPhaseCoulomb, 0,
            [&](int g) {
                return packed ? jk::coulomb_tiles((int)p[g].ndens, plans[g].f.slab)
                              : jk::cu_tiles((int)p[g].nao, (int)p[g].ndens);
            },
            all);
        if (packed)
            add(jk::kPhaseUnpackJ, 0, rows, all);
    }
    if (w & JK_WANT_K) {
        add(jk::kPhasePack, 0,
            [&](int g) { return jk::pack_tiles((int)p[g].nao, (int)p[g].ndens, (int)p[g].rank); }, all);
        if (mixed)
            add(jk::kPhaseMSliceC, 0, [&](int g) { return (plans[g].x.cp + 31) / 32; }, all);
        for (int c = 0; c < maxsteps; c++) {
            auto in_step = [&](int g) { return (i64)c * plans[g].f.qc < p[g].naux; };
            auto nq_of = [&](int g) {
                const i64 q0 = (i64)c * plans[g].f.qc;
                return (int)std::min<i64>(plans[g].f.qc, p[g].naux - q0);
            };
            if (mixed) {
                int nj = 1, maxnao = 1;
                for (int g = 0; g < G; g++) {
                    nj = std::max(nj, slicer_blocks(plans[g].x.kp));
                    maxnao = std::max(maxnao, (int)p[g].nao);
                }
                if (packed)      // bands of 8 rows through LDS; arg = 16 x LDS bytes + blocks
                    add(jk::kPhaseMSliceBPacked, c,
                        [&](int g) { return nq_of(g) * ((plans[g].x.mpb + 7) / 8); }, in_step,
                        16 * (int)sizeof(double) * 8 * maxnao + nj);
                else
                    add(jk::kPhaseMSliceB, c,
                        [&](int g) { return (int)(((i64)nq_of(g) * plans[g].x.mpb + 3) / 4); }, in_step,
                        nj);
                add(jk::kPhaseMHalf, c,
                    [&](int g) {
                        return jk::mixed_ht_tiles(plans[g].x.mpb,
                                                  plans[g].sym ? plans[g].x.cp_sym : plans[g].x.cp,
                                                  nq_of(g));
                    },
                    in_step);
                // one tile per (64-row block, key) of X/Y
                add(jk::kPhaseMRowmax, c,
                    [&](int g) {
                        const int nkey = plans[g].sym ? (int)p[g].ndens : 2 * (int)p[g].ndens;
                        return jk::cdiv_i(p[g].nao, 64) * nkey;
                    },
                    in_step);
                add(jk::kPhaseMSliceXY, c,
                    [&](int g) {
                        const int nkey = plans[g].sym ? (int)p[g].ndens : 2 * (int)p[g].ndens;
                        const int nkb = (int)(((i64)nq_of(g) * p[g].rank + 31) / 32);
                        return (int)(((i64)nkey * plans[g].x.mp + 31) / 32) * nkb;
                    },
                    in_step);
                add(jk::kPhaseMExchange, c,
                    [&](int g) {
                        return jk::mixed_ex_tiles(plans[g].x.mp, (int)p[g].ndens, plans[g].nsplit,
                                                  plans[g].sym);
                    },
                    in_step);
                continue;
            }
            // members whose plan chose 64 x 64 half-transform tiles get a launch of their own
            add(jk::kPhaseHalf, c,
                [&](int g) { return jk::ht_tiles((int)p[g].nao, (int)p[g].ndens, (int)p[g].rank, nq_of(g)); },
                [&](int g) { return in_step(g) && plans[g].tile == 0; });
            add(jk::kPhaseHalf64, c,
                [&](int g) { return jk::ht64_tiles((int)p[g].nao, (int)p[g].ndens, (int)p[g].rank, nq_of(g)); },
                [&](int g) { return in_step(g) && plans[g].tile == 1; });
            add(jk::kPhaseHalf16, c,
                [&](int g) {
                    const int R = (int)(p[g].ndens * p[g].rank);
                    return jk::ht_flat_tiles<jk::TileHalf16>((int)p[g].nao, plans[g].sym ? R : 2 * R,
                                                           nq_of(g));
                },
                [&](int g) { return in_step(g) && plans[g].tile == 4 && !packed; });
            add(jk::kPhaseHalf16Packed, c,
                [&](int g) {
                    const int R = (int)(p[g].ndens * p[g].rank);
                    return nq_of(g) * jk::cdiv_i(p[g].nao, jk::TileHalf16::BM) *
                           jk::cdiv_i(plans[g].sym ? R : 2 * R, jk::TileHalf16::BN);
                },
                [&](int g) { return in_step(g) && packed; });
            add(jk::kPhaseExchange, c,
                [&](int g) {
                    return plans[g].sym
                               ? plans[g].nsplit * (int)p[g].ndens * jk::ex_tri_tiles((int)p[g].nao)
                               : jk::ex_tiles((int)p[g].nao, (int)p[g].ndens, plans[g].nsplit);
                },
                in_step);
        }
        add(jk::kPhaseSum, 0, [&](int g) { return jk::sum_tiles(p[g].ndens * p[g].nao * p[g].nao); },
            [&](int g) { return plans[g].nsplit > 1; });
        add(jk::kPhaseMirror, 0, [&](int g) { return (int)p[g].ndens * jk::mirror_blocks((int)p[g].nao); },
            [&](int g) { return plans[g].sym != 0; });
    }
    // header: descriptors, then tables.  Its size is a bound that holds for
    // every pattern of symmetric members (the workspace query does not know
    // it): at most one more launch than the non-symmetric schedule, and at
    // most 2 G + 3 entries per table.
    Carve c;
    const size_t o_mem = c.take(sizeof(jk::BMember) * G);
    for (const Pending &L : pend) {
        const int n = (int)L.members.size();
        BLaunch bl;
        bl.phase = L.phase;
        bl.step = L.step;
        bl.arg = L.arg;
        bl.ntiles = 0;
        for (int t : L.tiles)
            bl.ntiles += t;
        bl.tab_off = o_mem + align_up(sizeof(jk::BMember) * G) + S.tabs.size() * sizeof(int);
        S.tabs.push_back(n);
        int acc = 0;
        for (int t : L.tiles) {
            S.tabs.push_back(acc);
            acc += t;
        }
        S.tabs.push_back(acc);
        for (int g : L.members)
            S.tabs.push_back(g);
        S.launches.push_back(bl);
    }
    size_t nlaunch_bound = 0;
    {
        // the non-symmetric schedule's launch count, plus the mirror launch
        // (J: four phases, six with packed B)
        const int per_step = mixed ? 5 : 4;
        nlaunch_bound = 6 + 2 + (size_t)maxsteps * per_step + 2;
    }
    c.take(sizeof(int) * std::max(S.tabs.size(), nlaunch_bound * (2 * (size_t)G + 3)));
    S.header_bytes = c.off;
    S.mem.resize(G);
    S.region.resize(G);
    for (int g = 0; g < G; g++) {
        S.region[g] = c.take(plans[g].total);
        jk::BMember &m = S.mem[g];
        memset(&m, 0, sizeof(m));
        m.npos = p[g].nao * p[g].nao;
        m.bslab = plans[g].f.slab;
        m.packed = plans[g].f.packed ? 1 : 0;
        m.nao = (int)p[g].nao;
        m.naux = (int)p[g].naux;
        m.nd = (int)p[g].ndens;
        m.r = (int)p[g].rank;
        m.qc = plans[g].f.qc;
        m.ldw = plans[g].f.ldw;
        m.nsplit = plans[g].nsplit;
        m.npb = plans[g].f.npb;
        m.plen = plans[g].f.plen;
        m.sym = plans[g].sym;
        if (mixed) {
            const MixPlan &x = plans[g].x;
            const int KB = jk::mixed_k_block();
            m.mp = x.mp;
            m.mpb = x.mpb;
            m.kp = x.kp;
            m.cp = x.cp;
            m.cpx = m.sym ? x.cp_sym : x.cp;
            m.bkb = (i64)x.f.qc * x.mpb * KB;
            m.bps = m.bkb * (x.kp / KB);
            m.ckb = (i64)x.cp * KB;
            m.cps = m.ckb * (x.kp / KB);
            m.xkb = (i64)2 * m.nd * x.mp * KB;
            m.xps = m.xkb * (x.jp / KB);
        }
    }
    S.total_bytes = c.off;
    // shape signature
    S.key.reserve(64 + 48 * G);
    for (int g = 0; g < G; g++) {
        char buf[160];
        snprintf(buf, sizeof buf, "%lld,%lld,%lld,%lld,%d,%d,%d,%d,%d;", (long long)p[g].nao,
                 (long long)p[g].naux, (long long)p[g].ndens, (long long)p[g].rank, p[g].precision,
                 p[g].flags, plans[g].f.qc, plans[g].tile, plans[g].sym);
        S.key += buf;
    }
    return S;
}

// Captured launch sequences, keyed by shape signature, workspace and device.
// At most kMaxGraphs are kept; inserting one more first destroys the oldest,
// after a synchronisation of the device it was made on (a replay of it may
// still be running).
constexpr size_t kMaxGraphs = 32;
struct GraphCache {
    std::mutex mu;
    struct Entry {
        hipGraphExec_t exec;
        int dev;
    };
    std::map<std::string, Entry> execs;
    std::vector<std::string> order;    // insertion order, oldest first
};
GraphCache &graph_cache()
{
    static GraphCache c;
    return c;
}

// Inserts exec under key (the cache mutex held); false if an eviction failed.
bool graph_cache_insert(GraphCache &gc, const std::string &key, hipGraphExec_t exec, int dev)
{
    while (gc.execs.size() >= kMaxGraphs && !gc.order.empty()) {
        const std::string old = gc.order.front();
        auto it = gc.execs.find(old);
        if (it != gc.execs.end()) {
            int cur = 0;
            if (hipGetDevice(&cur) != hipSuccess || hipSetDevice(it->second.dev) != hipSuccess)
                return false;
            const hipError_t e = hipDeviceSynchronize();
            (void)hipSetDevice(cur);
            if (e != hipSuccess)
                return false;
            (void)hipGraphExecDestroy(it->second.exec);
            gc.execs.erase(it);
        }
        gc.order.erase(gc.order.begin());
    }
    gc.execs[key] = GraphCache::Entry{exec, dev};
    gc.order.push_back(key);
    return true;
}

// Pinned host staging of the batched header, one buffer per device.  A call
// rewrites it only after the previous call's copy out of it has completed
// (an event recorded after that copy), so an asynchronous copy never reads a
// buffer that is being overwritten or freed.
struct HeaderStage {
    char *host = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;
};

hipError_t copy_header(const jk::BMember *mem, int nprob, const std::vector<int> &tabs,
                       size_t header_bytes, void *dst, hipStream_t s)
{
    static std::mutex mu;
    static std::map<int, HeaderStage> stages;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    std::lock_guard<std::mutex> lk(mu);
    HeaderStage &st = stages[dev];
    if (!st.done) {
        e = hipEventCreateWithFlags(&st.done, hipEventDisableTiming);
        if (e != hipSuccess) {
            st.done = nullptr;
            return e;
        }
    } else if ((e = hipEventSynchronize(st.done)) != hipSuccess) {
        return e;
    }
    if (st.cap < header_bytes) {
        if (st.host)
            (void)hipHostFree(st.host);
        st.host = nullptr;
        st.cap = 0;
        e = hipHostMalloc((void **)&st.host, header_bytes, hipHostMallocDefault);
        if (e != hipSuccess) {
            st.host = nullptr;
            return e;
        }
        st.cap = header_bytes;
    }
    memset(st.host, 0, header_bytes);
    memcpy(st.host, mem, sizeof(jk::BMember) * nprob);
    memcpy(st.host + align_up(sizeof(jk::BMember) * nprob), tabs.data(), sizeof(int) * tabs.size());
    e = hipMemcpyAsync(dst, st.host, header_bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess)
        return e;
    return hipEventRecord(st.done, s);
}

bool graphs_enabled()
{
    const char *e = getenv("JK_BATCHED_GRAPH");
    return !(e && e[0] == '0');
}

jk_status enqueue_batched(const BSchedule &S, char *ws, hipStream_t s)
{
    const jk::BMember *M = (const jk::BMember *)ws;
    for (const BLaunch &L : S.launches) {
        hipError_t e = jk::launch_batched_phase(L.phase, M, (const int *)(ws + L.tab_off), L.ntiles,
                                                L.step, s, L.arg);
        if (e != hipSuccess)
            return JK_EHIP;
    }
    return JK_OK;
}

jk_status build_batched(int32_t nprob, const jk_problem *p, const double *const *B,
                        const double *const *CL, const double *const *CR, double *const *J,
                        double *const *K, char *ws, hipStream_t s)
{
    const bool mixed = p[0].precision == JK_MIXED;
    std::vector<char> sym(nprob);
    for (int g = 0; g < nprob; g++)
        sym[g] = CL[g] == CR[g];
    BSchedule S = make_schedule(nprob, p, sym);
    // the header: descriptors with this call's pointers, then the tables
    for (int g = 0; g < nprob; g++) {
        jk::BMember &m = S.mem[g];
        const BPlan b = batched_plan(&p[g], sym[g] != 0);
        const FwdPlan &f = b.f;
        char *base = ws + S.region[g];
        m.B = B[g];
        m.CL = CL[g];
        m.CR = CR[g];
        m.J = J[g];
        m.K = K[g];
        m.Cc = (double *)(base + f.o_cc);
        m.D = (double *)(base + f.o_d);
        m.S = f.packed ? (double *)(base + f.o_s) : nullptr;
        m.part = (double *)(base + f.o_part);
        m.g = (double *)(base + f.o_g);
        m.goff = (long long)((S.region[g] + f.o_g) / sizeof(double));
        m.Xw = (double *)(base + f.o_x);
        m.Yw = (double *)(base + f.o_y);
        m.Kp = (double *)(base + (mixed ? b.x.o_kp : f.o_kp));
        if (mixed) {
            m.Bp = (int8_t *)(base + b.x.o_bp[0]);
            m.eB = (int *)(base + b.x.o_eb[0]);
            m.Cp = (int8_t *)(base + b.x.o_cp);
            m.eC = (int *)(base + b.x.o_ec);
            m.XY = (double *)(base + b.x.o_xy[0]);
            m.XYp = (int8_t *)(base + b.x.o_xyp[0]);
            m.eXY = (int *)(base + b.x.o_exy[0]);
            m.pm = (double *)(base + b.x.o_pm[0]);
        }
    }
    if (copy_header(S.mem.data(), nprob, S.tabs, S.header_bytes, ws, s) != hipSuccess)
        return JK_EHIP;

    if (jk::prepare_batched_kernels() != hipSuccess)
        return JK_EHIP;
    if (mixed && jk::prepare_batched_mixed_kernels() != hipSuccess)
        return JK_EHIP;
    if (s == nullptr || !graphs_enabled())
        return enqueue_batched(S, ws, s);

    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return JK_EHIP;
    char kbuf[64];
    snprintf(kbuf, sizeof kbuf, "|%p|%d", (void *)ws, dev);
    const std::string key = S.key + kbuf;
    GraphCache &gc = graph_cache();
    hipGraphExec_t exec = nullptr;
    {
        std::lock_guard<std::mutex> lk(gc.mu);
        auto it = gc.execs.find(key);
        if (it != gc.execs.end())
            exec = it->second.exec;
    }
    if (!exec) {
        hipGraph_t graph = nullptr;
        jk::ProfScope::set_capturing(true);
        if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            jk::ProfScope::set_capturing(false);
            return JK_EHIP;
        }
        jk_status st = enqueue_batched(S, ws, s);
        hipError_t e = hipStreamEndCapture(s, &graph);
        jk::ProfScope::set_capturing(false);
        if (st != JK_OK || e != hipSuccess)
            return JK_EHIP;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess)
            return JK_EHIP;
        std::lock_guard<std::mutex> lk(gc.mu);
        if (!graph_cache_insert(gc, key, exec, dev)) {
            (void)hipGraphExecDestroy(exec);
            return JK_EHIP;
        }
    }
    return hipGraphLaunch(exec, s) == hipSuccess ? JK_OK : JK_EHIP;
}

} // namespace

extern "C" {

size_t jk_workspace_bytes(const jk_problem *p)
{
    if (!valid_problem(p))
        return 0;
    return std::max(forward_bytes(p), plan_vjp(p).total);
}

static jk_status jk_build_impl(const jk_problem *p, const double *B, const double *CL, const double *CR,
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
    return build_plain(p, B, CL, CR, J, K, (char *)ws, (hipStream_t)stream);
}

jk_status jk_build(const jk_problem *p, const double *B, const double *CL, const double *CR,
                   double *J, double *K, void *ws, size_t ws_bytes, void *stream)
{
    try {
        return jk_build_impl(p, B, CL, CR, J, K, ws, ws_bytes, stream);
    } catch (...) {
        return JK_ENOMEM;
    }
}

size_t jk_slices_bytes(const jk_problem *p)
{
    if (!valid_problem(p) || p->precision != JK_MIXED)
        return 0;
    return slice_layout(p).total;
}

static jk_status jk_slice_b_impl(const jk_problem *p, const double *B, void *slices,
                                 size_t slices_bytes, void *stream)
{
    if (!valid_problem(p) || p->precision != JK_MIXED || !B || !slices ||
        ((uintptr_t)slices) % kAlign)
        return JK_EINVAL;
    if (slices_bytes < jk_slices_bytes(p))
        return JK_EWORKSPACE;
    if (p->nslice != 0 && p->nslice != jk::mixed_nslice())
        return JK_EUNSUPPORTED;
    const SliceLayout L = slice_layout(p);
    const int KB = jk::mixed_k_block();
    const int nao = (int)p->nao, naux = (int)p->naux;
    if (packed_b(p) && !jk::mixed_packed_ok(nao, L.kp))
        return JK_EUNSUPPORTED;
    char *base = (char *)slices;
    int8_t *planes = (int8_t *)(base + L.o_planes);
    int *exps = (int *)(base + L.o_exp);
    hipStream_t s = (hipStream_t)stream;
    if (packed_b(p))
        JK_TRY(jk::launch_slice_b_packed(B, jk::pk_size(nao), naux, nao, L.mp, L.kp / KB, planes,
                                         L.pstride, L.kbstride, exps, s));
    else
        JK_TRY(jk::launch_slice_b(B, (i64)nao * nao, nao, naux, nao, nao, L.mp, L.kp / KB, planes,
                                  L.pstride, L.kbstride, exps, s));
    return JK_OK;
}

jk_status jk_slice_b(const jk_problem *p, const double *B, void *slices, size_t slices_bytes,
                     void *stream)
{
    try {
        return jk_slice_b_impl(p, B, slices, slices_bytes, stream);
    } catch (...) {
        return JK_ENOMEM;
    }
}

static jk_status jk_build_sliced_impl(const jk_problem *p, const double *B, const void *slices,
                                      size_t slices_bytes, const double *CL, const double *CR,
                                      double *J, double *K, void *ws, size_t ws_bytes, void *stream)
{
    if (!valid_problem(p) || p->precision != JK_MIXED)
        return JK_EINVAL;
    const int w = want(p);
    if (!B || !CL || !CR || !ws || !slices || ((uintptr_t)slices) % kAlign)
        return JK_EINVAL;
    if ((w & JK_WANT_J) && !J)
        return JK_EINVAL;
    if ((w & JK_WANT_K) && !K)
        return JK_EINVAL;
    if (((uintptr_t)ws) % kAlign)
        return JK_EINVAL;
    if (slices_bytes < jk_slices_bytes(p))
        return JK_EWORKSPACE;
    if (ws_bytes < jk_workspace_bytes(p))
        return JK_EWORKSPACE;
    const KSeg seg{B, (int)p->naux, 1.0};
    BuildOut o;
    o.J = J;
    o.K = K;
    return build_mixed(p, B, &seg, 1, CL, CR, o, (char *)ws, (hipStream_t)stream,
                       (const char *)slices);
}

jk_status jk_build_sliced(const jk_problem *p, const double *B, const void *slices,
                          size_t slices_bytes, const double *CL, const double *CR, double *J,
                          double *K, void *ws, size_t ws_bytes, void *stream)
{
    try {
        return jk_build_sliced_impl(p, B, slices, slices_bytes, CL, CR, J, K, ws, ws_bytes, stream);
    } catch (...) {
        return JK_ENOMEM;
    }
}

} // extern "C"

namespace {

// Device address of the scratch array on the current device, looked up once
// per device (with that device current) and kept.
hipError_t scratch_address(char **out)
{
    static std::mutex mu;
    static std::map<int, char *> addr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    std::lock_guard<std::mutex> lk(mu);
    auto it = addr.find(dev);
    if (it == addr.end()) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        if (ptr == nullptr || ((uintptr_t)ptr) % kAlign)
            return hipErrorInvalidSymbol;
        it = addr.emplace(dev, (char *)ptr).first;
    }
    *out = it->second;
    return hipSuccess;
}

// Largest chunk budget (MiB, a power of two up to 256) whose FP64 plan fits
// the scratch array; 0 if none does.
int noalloc_chunk_mb(const jk_problem *p)
{
    for (int mb = 256; mb >= 1; mb /= 2)
        if (plan_forward(p, (size_t)mb << 20).total <= kNoAllocScratchBytes)
            return mb;
    return 0;
}

jk_status jk_build_noalloc_impl(const jk_problem *p, const double *B, const double *CL,
                                const double *CR, double *J, double *K, void *stream)
{
    if (!valid_problem(p))
        return JK_EINVAL;
    const int w = want(p);
    if (!B || !CL || !CR)
        return JK_EINVAL;
    if ((w & JK_WANT_J) && !J)
        return JK_EINVAL;
    if ((w & JK_WANT_K) && !K)
        return JK_EINVAL;
    if (p->precision != JK_FP64)
        return JK_EUNSUPPORTED;
    const int mb = noalloc_chunk_mb(p);
    if (mb == 0)
        return JK_EWORKSPACE;
    char *ws = nullptr;
    if (scratch_address(&ws) != hipSuccess)
        return JK_EHIP;
    // the recorded tile, with the chunk budget the scratch array allows
    jk_tuning plan = plan_tuning(p);
    plan.chunk_mb = mb;
    t_forced = &plan;
    const jk_status st = build_plain(p, B, CL, CR, J, K, ws, (hipStream_t)stream);
    t_forced = nullptr;
    return st;
}

} // namespace

extern "C" {

jk_status jk_build_noalloc(const jk_problem *p, const double *B, const double *CL, const double *CR,
                           double *J, double *K, void *stream)
{
    try {
        return jk_build_noalloc_impl(p, B, CL, CR, J, K, stream);
    } catch (...) {
        t_forced = nullptr;
        return JK_ENOMEM;
    }
}

size_t jk_fock_workspace_bytes(const jk_problem *p, int64_t naux_lr)
{
    if (!valid_problem(p) || naux_lr < 0 || naux_lr > ((int64_t)1 << 28))
        return 0;
    return forward_bytes(p);
}

static jk_status jk_fock_impl(const jk_problem *p, const double *B, const double *B_lr, int64_t naux_lr,
                  const double *CL, const double *CR, const double *coef, double *F, void *ws,
                  size_t ws_bytes, void *stream)
{
    if (!valid_problem(p) || want(p) != (JK_WANT_J | JK_WANT_K))
        return JK_EINVAL;
    if (!B || !CL || !CR || !coef || !F || !ws || ((uintptr_t)ws) % kAlign)
        return JK_EINVAL;
    for (int i = 0; i < 3; i++)
        if (!std::isfinite(coef[i]))
            return JK_EINVAL;
    if ((B_lr == nullptr) != (naux_lr == 0) || (B_lr == nullptr && coef[2] != 0.0))
        return JK_EINVAL;
    if (naux_lr < 0 || naux_lr > ((int64_t)1 << 28))
        return JK_EINVAL;
    if (ws_bytes < jk_fock_workspace_bytes(p, naux_lr))
        return JK_EWORKSPACE;
    KSeg seg[2];
    int nseg = 0;
    if (coef[1] != 0.0)
        seg[nseg++] = KSeg{B, (int)p->naux, coef[1]};
    if (B_lr && coef[2] != 0.0)
        seg[nseg++] = KSeg{B_lr, (int)naux_lr, coef[2]};
    BuildOut o;
    o.F = F;
    o.cj = coef[0];
    return p->precision == JK_MIXED
               ? build_mixed(p, B, seg, nseg, CL, CR, o, (char *)ws, (hipStream_t)stream)
               : build_fp64(p, B, seg, nseg, CL, CR, o, (char *)ws, (hipStream_t)stream);
}

jk_status jk_fock(const jk_problem *p, const double *B, const double *B_lr, int64_t naux_lr,
                  const double *CL, const double *CR, const double *coef, double *F, void *ws,
                  size_t ws_bytes, void *stream)
{
    try {
        return jk_fock_impl(p, B, B_lr, naux_lr, CL, CR, coef, F, ws, ws_bytes, stream);
    } catch (...) {
        return JK_ENOMEM;
    }
}

static size_t jk_batched_workspace_bytes_impl(int32_t nprob, const jk_problem *p)
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
    // every member owns its plan's workspace, plus the header (the mixed form
    // falls back to one build after another, in a single-build workspace,
    // when a member's rows are too long for the batched slicer)
    if (p[0].precision == JK_FP64 || batched_mixed_ok(nprob, p)) {
        size_t t = make_schedule(nprob, p, std::vector<char>()).total_bytes;
        return t > mx ? t : mx;
    }
    return mx;
}

size_t jk_batched_workspace_bytes(int32_t nprob, const jk_problem *p)
{
    try {
        return jk_batched_workspace_bytes_impl(nprob, p);
    } catch (...) {
        return 0;
    }
}

static jk_status jk_build_batched_impl(int32_t nprob, const jk_problem *p, const double *const *B,
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
    if (p[0].precision == JK_FP64 || batched_mixed_ok(nprob, p))
        return build_batched(nprob, p, B, CL, CR, J, K, (char *)ws, (hipStream_t)stream);
    for (int32_t g = 0; g < nprob; g++) {
        jk_status st = build_plain(&p[g], B[g], CL[g], CR[g], J[g], K[g], (char *)ws,
                                   (hipStream_t)stream);
        if (st != JK_OK)
            return st;
    }
    return JK_OK;
}

jk_status jk_build_batched(int32_t nprob, const jk_problem *p, const double *const *B,
                           const double *const *CL, const double *const *CR, double *const *J,
                           double *const *K, void *ws, size_t ws_bytes, void *stream)
{
    try {
        return jk_build_batched_impl(nprob, p, B, CL, CR, J, K, ws, ws_bytes, stream);
    } catch (...) {
        return JK_ENOMEM;
    }
}

static jk_status jk_autotune_impl(const jk_problem *p, const double *B, const double *CL, const double *CR,
                      double *J, double *K, void *ws, size_t ws_bytes, void *stream,
                      int32_t reps, jk_tuning *chosen)
{
    if (!valid_problem(p) || reps < 0 || reps > 100)
        return JK_EINVAL;
    const int w = want(p);
    if (!B || !CL || !CR || !ws || ((uintptr_t)ws) % kAlign)
        return JK_EINVAL;
    if (((w & JK_WANT_J) && !J) || ((w & JK_WANT_K) && !K))
        return JK_EINVAL;
    if (ws_bytes < jk_workspace_bytes(p))
        return JK_EWORKSPACE;
    if (reps == 0)
        reps = 2;
    hipStream_t s = (hipStream_t)stream;
    std::vector<jk_tuning> cand;
    // FP64 half-transform tiles: the 16 x 16 x 4 engine's two (4, 3) and the
    // eight-wave tile of the 4x4x4 engine (2); other precisions and layouts
    // have one kernel
    std::vector<int> tiles = {4};
    if (p->precision == JK_FP64 && !packed_b(p))
        tiles = {4, 3, 2};
    for (int tile : tiles)
        for (int mb : {128, 256, 512, 1024, 2048, 4096})
            cand.push_back(jk_tuning{tile, mb});
    TimedEvents E;
    JK_TRY(E.create());
    float best = 0.0f;
    jk_tuning pick = cand[0];
    for (size_t c = 0; c < cand.size(); c++) {
        t_forced = &cand[c];
        jk_status st = build_plain(p, B, CL, CR, J, K, (char *)ws, s);
        hipError_t he = hipEventRecord(E.ev[0], s);
        for (int i = 0; i < reps && st == JK_OK && he == hipSuccess; i++)
            st = build_plain(p, B, CL, CR, J, K, (char *)ws, s);
        t_forced = nullptr;
        if (st != JK_OK)
            return st;
        JK_TRY(he);
        JK_TRY(hipEventRecord(E.ev[1], s));
        JK_TRY(hipEventSynchronize(E.ev[1]));
        float ms = 0.0f;
        JK_TRY(hipEventElapsedTime(&ms, E.ev[0], E.ev[1]));
        if (c == 0 || ms < best) {
            best = ms;
            pick = cand[c];
        }
    }
    jk::tuning_record(p, pick);
    if (chosen)
        *chosen = pick;
    return build_plain(p, B, CL, CR, J, K, (char *)ws, s);
}

jk_status jk_autotune(const jk_problem *p, const double *B, const double *CL, const double *CR,
                      double *J, double *K, void *ws, size_t ws_bytes, void *stream,
                      int32_t reps, jk_tuning *chosen)
{
    try {
        return jk_autotune_impl(p, B, CL, CR, J, K, ws, ws_bytes, stream, reps, chosen);
    } catch (...) {
        return JK_ENOMEM;
    }
}

static jk_status jk_vjp_impl(const jk_problem *p, const double *B, const double *CL, const double *CR,
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
    // stages C and D read a slab's block [P' | R'] (nao x 2R) through one buffer
    // resource, whose offsets stop at 4 GiB
    if (!jk::buf_extent_ok(p->nao * 2 * p->ndens * p->rank))
        return JK_EUNSUPPORTED;
    if (!dB && !dCL)
        return JK_OK;
    return vjp_fp64(p, B, CL, CR, Jbar, Kbar, dB, dCL, dCR, (char *)ws, (hipStream_t)stream);
}

jk_status jk_vjp(const jk_problem *p, const double *B, const double *CL, const double *CR,
                 const double *Jbar, const double *Kbar, double *dB, double *dCL, double *dCR,
                 void *ws, size_t ws_bytes, void *stream)
{
    try {
        return jk_vjp_impl(p, B, CL, CR, Jbar, Kbar, dB, dCL, dCR, ws, ws_bytes, stream);
    } catch (...) {
        return JK_ENOMEM;
    }
}

static jk_status jk_plan_describe_impl(const jk_problem *p, const jk_tuning *t, jk_plan_info *out)
{
    if (!valid_problem(p) || !out)
        return JK_EINVAL;
    const jk_tuning tu = t ? *t : plan_tuning(p);
    if (tu.ht_tile < 0 || tu.ht_tile > 4 || tu.chunk_mb < 64 || tu.chunk_mb > 4096)
        return JK_EINVAL;
    const size_t budget = (size_t)tu.chunk_mb << 20;
    memset(out, 0, sizeof(*out));
    if (p->precision == JK_MIXED) {
        const MixPlan x = plan_mixed(p, budget);
        const int KB = jk::mixed_k_block();
        const int nkb = x.jp / KB;
        out->chunk_slabs = x.f.qc;
        out->nsplit = x.nsplit;
        out->nsplit_sym = x.nsplit_sym;
        const int ns = std::min(x.nsplit, x.nsplit_sym);
        const int ex_depth = (nkb + ns - 1) / ns * KB;
        out->int_depth = std::max(x.kp, ex_depth);
        out->int_depth_cap = jk::mixed_max_depth();
    } else {
        const FwdPlan f = plan_forward(p, budget);
        out->chunk_slabs = f.qc;
        out->nsplit = f.nsplit;
        out->nsplit_sym = f.nsplit_sym;
    }
    return JK_OK;
}

jk_status jk_plan_describe(const jk_problem *p, const jk_tuning *t, jk_plan_info *out)
{
    try {
        return jk_plan_describe_impl(p, t, out);
    } catch (...) {
        return JK_ENOMEM;
    }
}

const char *jk_status_str(jk_status s)
{
    // A C caller may pass any int; read it as one (a load of an enum object
    // outside the enumerators' range is undefined in C++).
    int v = 0;
    std::memcpy(&v, &s, sizeof v < sizeof s ? sizeof v : sizeof s);
    switch (v) {
    case JK_OK: return "ok";
    case JK_EINVAL: return "invalid argument";
    case JK_EWORKSPACE: return "workspace too small";
    case JK_EUNSUPPORTED: return "unsupported combination";
    case JK_EHIP: return "HIP launch or runtime failure";
    case JK_ENOMEM: return "host allocation failed";
    }
    return "unknown status";
}

} // extern "C"

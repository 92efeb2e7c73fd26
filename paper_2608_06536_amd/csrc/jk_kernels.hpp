// jk_kernels.hpp -- launchers of the device kernels (internal to the library).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace jk {

typedef int64_t i64;

// Brackets one kernel launch with timing events when jk_prof_enable is on
// (include/jk_prof.h); does nothing otherwise.
class ProfScope {
  public:
    ProfScope(const char *name, hipStream_t s);
    ~ProfScope();
    // While a stream is being captured into a graph no events are recorded.
    static void set_capturing(bool on);
    ProfScope(const ProfScope &) = delete;
    ProfScope &operator=(const ProfScope &) = delete;

  private:
    hipStream_t stream_;
    int pair_;
};

// Workgroup slots of the current device for two resident workgroups per CU.
int device_slots();
// Split count s in [1, smax] for a grid of tiles * s workgroups: the smallest s
// whose last round of workgroups is at least 90% full with at least one full
// round, else the s with the fullest rounds.
int pick_split(int tiles, int smax);
// Allows `bytes` of dynamic LDS for kernel fn on the current device (once per
// kernel and device).
hipError_t set_dynamic_lds(const void *fn, int bytes);
// Same with an explicit number of concurrent workgroup slots.
int pick_split_slots(int tiles, int smax, int slots);

hipError_t launch_pack_c(const double *CL, const double *CR, double *Cc, int nao, int nd, int r,
                         hipStream_t s);
hipError_t launch_density(const double *CL, const double *CR, double *D, int nao, int nd, int r,
                          hipStream_t s);
int project_nblocks(int64_t npos, int naux, int nd, int *plen);
// 9 to 16 matrices A_k (contiguous, npos apart) projected in one pass over B
// into g[k][Q]; part holds project16_nblocks x naux x 16 doubles.
int project16_nblocks(int64_t npos, int naux, int *plen);
hipError_t launch_project16(const double *B, const double *A, double *part, double *g, int naux,
                            int nd, int64_t npos, hipStream_t s);
hipError_t launch_project(const double *B, const double *A, double *part, double *g, int naux,
                          int nd, int64_t npos, hipStream_t s);
// J (+)= scale * sum_Q g B^Q; accumulate adds to what J holds.
hipError_t launch_coulomb(const double *B, const double *g, double *J, int naux, int nd,
                          int64_t npos, hipStream_t s, double scale = 1.0, int accumulate = 0);
// Full-square symmetric slabs read on their upper triangles (half the bytes
// of B).  fold_upper: A_k[m][n] += A_k[n][m], A_k[n][m] = 0 for n > m, in
// place (nmat matrices).  project_upper: g[k][Q] = <B^Q, A_k> from the folded
// A; part holds project_upper_blocks pairs x naux x (8 groups, or 16) doubles;
// sixteen: 9 to 16 matrices in one pass (else groups of 8).
hipError_t launch_fold_upper(double *A, int nao, int nmat, hipStream_t s);
int project_upper_blocks(int nao, int naux, int nkg, int *G);
hipError_t launch_project_upper(const double *B, const double *S, double *part, double *g, int nao,
                                int naux, int nd, hipStream_t s, bool sixteen = false);
// J (bit-identical to launch_coulomb's for symmetric slabs).
hipError_t launch_coulomb_upper(const double *B, const double *g, double *J, int nao, int naux,
                                int nd, hipStream_t s, double scale = 1.0, int accumulate = 0);
// packed: B holds packed upper-triangle slabs (nao (nao + 1) / 2 doubles).
// tile (full slabs only; jk_tune.h): 0 = 128 x 64 workgroup tiles of four
// waves, 1 = 64 x 64, 2 = 128 x 64 of eight waves (4x4x4 engine); 3 = 128 x 128,
// 4 = 128 x 64 over stacked slabs (16x16x4 engine).  prof: the name the
// launch is timed under.
hipError_t launch_half_transform(const double *B, const double *Cc, double *Xw, double *Yw,
                                 int nao, int nd, int r, int q0, int nq, int ldw, hipStream_t s,
                                 int ncol = -1, int packed = 0, int tile = 0,
                                 const char *prof = "half_transform");
// S_k = D_k + D_k^T off the diagonal, D_k on it, as packed upper triangles.
hipError_t launch_sym_pack(const double *D, double *S, int nao, int nd, hipStream_t s);
// out_k (+)= scale * P_k, P_k a packed symmetric matrix, written in full.
hipError_t launch_unpack_sym(const double *P, double *out, int nao, int nd, double scale,
                             int accumulate, hipStream_t s);
// Lower triangle of every K_k from its upper triangle.
hipError_t launch_mirror_upper(double *K, int nao, int nd, hipStream_t s);
int exchange_nsplit(int nao, int nd, int nj, int sym = 0);
// Every chunk's contribution is multiplied by scale before it is stored or
// added (scale 1 leaves it unchanged bit for bit).
hipError_t launch_exchange(const double *Xw, const double *Yw, double *Kp, int nao, int nd, int nj,
                           int ldw, int nsplit, int accumulate, hipStream_t s, int sym = 0,
                           double scale = 1.0);
hipError_t launch_sum_splits(const double *part, double *out, i64 n, int nsplit, hipStream_t s);

// derivative (jk_vjp.hip)
hipError_t launch_omega_expand(const double *om, double *omx, int naux, int nd, int r,
                               hipStream_t s);
// One of the two stage-B products: which = 0 gives P' (Zw = Y_ws), 1 gives R' (Zw = X_ws).
hipError_t launch_vjp_stage_b_one(int which, const double *V, const double *Zw, const double *Cc,
                                  const double *omx, double *L, int nao, int nd, int r, int q0,
                                  int nj, int ldw, int has_v, int has_w, hipStream_t s);
hipError_t launch_vjp_stage_b(const double *V, const double *Xw, const double *Yw,
                              const double *Cc, const double *omx, double *L, int nao, int nd,
                              int r, int q0, int nj, int ldw, int has_v, int has_w, hipStream_t s);
int vjp_stage_c_nsplit(int nao, int R, int qc);
hipError_t launch_vjp_stage_c(const double *B, const double *L, double *dCp, int nao, int R,
                              int q0, int nq, int nsplit, int accumulate, hipStream_t s);
hipError_t launch_vjp_dc_finish(const double *dCp, double *dCL, double *dCR, int nao, int nd,
                                int r, int nsplit, hipStream_t s);
hipError_t launch_vjp_e_matrix(const double *D, double *E, int nao, int nd, hipStream_t s);
hipError_t launch_vjp_stage_d(const double *L, const double *Cc, double *dB, int nao, int R,
                              int q0, int nq, hipStream_t s);
// Packed B (jk.h JK_B_PACKED): full squares of slabs q0 .. q0 + nq - 1 into
// out[nq][nao][nao]; stage D writing the packed gradient of those slabs
// (dB[a][b] + dB[b][a] for a < b, dB[a][a] on the diagonal).
hipError_t launch_unpack_slabs(const double *Bp, double *out, int nao, int q0, int nq,
                               hipStream_t s);
hipError_t launch_vjp_stage_d_packed(const double *L, const double *Cc, double *dB, int nao, int R,
                                     int q0, int nq, hipStream_t s);
hipError_t launch_vjp_db_affine(const double *gam, const double *om, const double *W,
                                const double *E, double *dB, int nd, int naux, i64 npos, int q0,
                                int nq, hipStream_t s);

// mixed precision (jk_mixed.hip)
int mixed_nslice();
int mixed_row_pad();
// rows per slab of B's digit planes (a multiple of the INT8 half-transform's
// row tile; X/Y planes keep mixed_row_pad)
int mixed_b_row_pad();
int mixed_k_pad();
int mixed_k_block();
hipError_t launch_slice_rows(const double *src, i64 bs, i64 rs, i64 ks, int nb, int nr, int nk,
                             int rp, int nkb, int8_t *out, i64 pstride, i64 kbstride, int *exps,
                             hipStream_t s);
hipError_t launch_slice_b(const double *src, i64 bs, i64 rs, int nb, int nr, int nk, int rp, int nkb,
                          int8_t *out, i64 pstride, i64 kbstride, int *exps, hipStream_t s);
// widths 2 nd r of X/Y the mixed path takes
int mixed_rowmax_ok(int R2);
hipError_t launch_slice_xy(const double *XY, int nao, int nkey, int r, int mp, int nj, int nkb,
                           int8_t *out, i64 pstride, i64 kbstride, const int *exps, hipStream_t s);
// pm (optional): the row maxima of the chunk's X and Y per tile
// (xy_rowmax_pm_doubles doubles), reduced into exponents by launch_xy_rowmax_pm.
hipError_t launch_ht_mixed(const int8_t *Bp, i64 bpstride, i64 bkbstride, const int *eB,
                           const int8_t *Cp, i64 cpstride, i64 ckbstride, const int *eC, double *XY,
                           int nao, int R2, int nq, int mp, int cp, int nkb, hipStream_t s,
                           double *pm = nullptr, int r = 1);
int xy_rowmax_slots(int r, int nkey);
size_t xy_rowmax_pm_doubles(int nq, int mp, int cp, int r, int nkey);
// pm rows mp per slab (the half-transform's row pitch); exps[key mpe + m]
hipError_t launch_xy_rowmax_pm(const double *pm, int nao, int nq, int nkey, int r, int mp, int mpe,
                               int cp, int *exps, hipStream_t s);
// Exchange splits of a chunk of nkb inner blocks: chosen for occupancy, and
// never fewer than keep each split's int32 sums exact (mixed_max_depth()
// inner indices at most).
int ex_mixed_nsplit(int mp, int nd, int nkb, int sym = 0);
int mixed_max_depth();
// Workgroups of the mixed half-transform of nq slabs (cpx padded factor
// columns) and of the mixed exchange with nsplit splits.
int mixed_ht_tiles(int mp, int cpx, int nq);
int mixed_ex_tiles(int mp, int nd, int nsplit, int sym);
// B digit planes from packed slabs (slab stride bs = nao (nao + 1) / 2);
// mixed_packed_ok tells whether the packed slicer covers rows of kp inner
// elements (kp <= 2048).
hipError_t launch_slice_b_packed(const double *src, i64 bs, int nb, int nao, int rp, int nkb,
                                 int8_t *out, i64 pstride, i64 kbstride, int *exps, hipStream_t s);
int mixed_packed_ok(int nao, int kp);
hipError_t launch_ex_mixed(const int8_t *Xp, const int8_t *Yp, i64 pstride, i64 kbstride,
                           const int *eX, const int *eY, double *Kp, int nao, int nd, int mp, int nkb,
                           int nsplit, int accumulate, hipStream_t s, int sym = 0,
                           double scale = 1.0);

} // namespace jk

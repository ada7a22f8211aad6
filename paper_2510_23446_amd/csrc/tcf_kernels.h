// Host launch wrappers of the libtcf kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "tcf_device.h"

namespace tcf {

void launch_tables(const DevPatch* P, int np, const double* gx, const double* gw, double* tabs,
                   double* ptab, hipStream_t st);
template <class T>
void launch_assemble(const DevPatch* P, const int* col_prefix, int np, int total_cols,
                     const int* r_loc, const double* tabs, double dt, T* A, hipStream_t st);
void launch_wapply(const DevPatch* P, const int* plist, const int* row_prefix, int nlist,
                   int total_rows, int nrhs, const int* r_loc, const int* loc2r,
                   const double* tabs, double dt, int mass_only, const double* x, double* y,
                   int64_t ldv, hipStream_t st);
void launch_load_batch(const DevPatch* P, const LoadJob* jobs, const int* prefix, int njobs,
                       int total, int nrhs, const int* r_loc, const double* ptab, const double* F,
                       int vec, double* out, int64_t ldv, hipStream_t st);
template <class T>
void launch_potrf(const FactorJob* jobs, int njobs, int k, T* A, int* fail, hipStream_t st);
template <class T>
void launch_trsm_panel(const FactorJob* jobs, const int* prefix, int njobs, int total, int k, T* A,
                       hipStream_t st);
template <class T>
void launch_syrk(const FactorJob* jobs, const int* prefix, int njobs, int total, int k, int mode,
                 T* A, hipStream_t st);
int syrk_super_panel();
template <class T>
void launch_copy_sbb(const DevPatch* P, const int* prefix, int np, int total, const T* A, T* S,
                     hipStream_t st);
template <class T>
void launch_fill_G(const DevPatch* P, const int* prefix, int np, int total, const T* A, T* G,
                   hipStream_t st);
template <class T>
void launch_fill_Q(const DevPatch* P, const int* prefix, int np, int total, const T* A, T* Q,
                   hipStream_t st);
template <class T>
void launch_coarse_add(const DevPatch* P, int s, int n_p, const int* p_rank, const T* A,
                       double* SPi, int ldc, hipStream_t st);
void launch_identity_pad(double* M, int ld, int n0, int n, hipStream_t st);
template <class T>
void launch_trsm_dinv(const TrsmJob* jobs, const int* dprefix, int njobs, int total, const T* L,
                      T* D, hipStream_t st);
int trsm_rl_panel();
template <class T>
void launch_trsm_rl_diag(const TrsmJob* jobs, const int* cprefix, const int* dprefix, int njobs,
                         int total, int s, int fwd, const T* L, const T* D, T* B, hipStream_t st);
template <class T>
void launch_trsm_rl_update(const TrsmJob* jobs, const int* tprefix, int njobs, int total, int s,
                           int fwd, const T* L, T* B, hipStream_t st);
template <class T>
void launch_dotcols(const DotJob* jobs, const int* prefix, int njobs, int total, int max_rows,
                    const T* M, int xmode, const double* xv, const int* gidx,
                    const signed char* gsgn, double xscale, double* out, const int* done,
                    hipStream_t st);
template <class T>
void launch_axpyrows(const AxpyJob* jobs, const int* prefix, int njobs, int total, int max_cols,
                     const T* M, const double* yv, const int* yidx, const double* base,
                     const int* base_off, double alpha, double* out, int tri_cols,
                     const int* done, hipStream_t st);
template <class T>
void launch_condense(const DevPatch* P, const int* plist, const int* prefix, int nlist, int total,
                     int nrhs, int max_ni, const T* Q, const double* f, double* ygg, int64_t ldv,
                     hipStream_t st);
// The condensation and the interior recovery for R <= 32 columns at once
// (matrix cores); prefixes over ceil(n_r / 64) resp. ceil(n_i / 64) blocks.
template <class T>
void launch_condense_w(const DevPatch* P, const int* plist, const int* prefix, int nlist,
                       int total, int R, const T* Q, const double* f, double* ygg, int64_t ldv,
                       hipStream_t st);
template <class T>
void launch_qapply_w(const DevPatch* P, const int* plist, const int* prefix, int nlist, int total,
                     int R, const T* Q, const double* z, double* out, int64_t ldv,
                     hipStream_t st);
void launch_jump(int n, const int* pp, const int* pm, const double* w, double scale, double* y,
                 const double* dotw, double* partial, const int* done, hipStream_t st);
void launch_coarse_gather(int n, const int* ptr, const int* ia, const double* srcA, double sa,
                          const int* ib, const double* srcB, double sb, const double* extra,
                          double* out, const int* done, hipStream_t st);
void launch_rowdot(int n, int nb, const double* rows, int64_t ld, const double* v, double* c,
                   const double* a, const double* b, int extra, hipStream_t st);
void launch_multiaxpy(int n, int nb, const double* c, double sgn, const double* X, const double* FX,
                      int64_t ld, double* v, double* Fv, hipStream_t st);
void launch_store_dir(int n, const double* nu2, const double* ref, double tol, const double* v,
                      const double* Fv, double* x, double* fx, hipStream_t st);
void launch_copy_sub(int n, const double* a, const double* b, const double* c, double* v,
                     double* w, hipStream_t st);
template <class T>
void launch_diag_range(const DevPatch* P, int np, const T* A, double* out, hipStream_t st);
void launch_axpby(int64_t n, double alpha, const double* x, double beta, double* y,
                  hipStream_t st);
void launch_sub_gather(int n, const int* ia, const double* a, const int* ib, const double* b,
                       double* out, hipStream_t st);
void launch_scatter(int n, const int* dst, const int* sidx, const double* src, double scale,
                    double* out, const int* done, hipStream_t st);
void launch_to_global(int64_t n, const int64_t* gid, const double* a, double* out,
                      hipStream_t st);

}  // namespace tcf

namespace tcf {
void launch_build_z(int64_t n, const signed char* is_int, const double* y, const double* a,
                    double* zr, hipStream_t st);
}  // namespace tcf
namespace tcf {
void launch_asm_norm2(int n, const int* ptr, const int* idx, const double* x, int first_copy,
                      double* partial, double* out, hipStream_t st);
}  // namespace tcf
namespace tcf {
void launch_to_float(int64_t n, const double* a, float* b, hipStream_t st);
}  // namespace tcf
namespace tcf {
void launch_residual(const DevPatch* P, const int* plist, const int* row_prefix, int nlist,
                     int total_rows, const int* r_loc, const int* loc2r, const double* tabs,
                     double dt, const double* f, const double* x, double* r, hipStream_t st);
}  // namespace tcf
namespace tcf {
void launch_jump_add(int n, const int* pp, const int* pm, const double* a, double scale, double* y,
                     hipStream_t st);
}  // namespace tcf
namespace tcf {
void launch_assemble_split(int n, const int* ptr, const int* idx, double* x, hipStream_t st);
}  // namespace tcf
namespace tcf {
// Row-panel tiles in the matrix cores' operand order (k_pack_panel).
template <class TS, class TD>
void launch_pack_panel(const PackJob* jobs, int njobs, const TS* src, TD* dst, hipStream_t st);
template <class TS, class TD>
void launch_pack_tiles(const PackJob* jobs, int njobs, const TS* src, TD* dst, hipStream_t st);
template <class T>
// group: 0 F apply, 2 preconditioner (signed gather inputs), 1 Phi_b N q
// and 4 coarse factor sweeps (plain gather), 3 coarse top block (direct
// inputs)
// R (1..4) right-hand sides at once: inputs xv[j * xld + i], outputs
// y[j * yld + i], quadratic-form slots qslot[j * TCF_QSLOTS + k].
void launch_tiles(int group, int R, const TileJob* jobs, int njobs, const T* M, const double* xv,
                  int xld, const int* gidx, const double* gsgn, double scale, double* y,
                  int yld, const int* ymap, double* qslot, const int* done, hipStream_t st);
// Row panels on the matrix cores (R <= 32 right-hand sides): group names
// the operator as for launch_tiles; groups 0 to 3 read their inputs
// directly, xv[j * xld + i] (gathered beforehand by launch_gather_cols),
// group 4 (the coarse factor's sweeps) through gidx.  A job owns its
// output rows (y[j * yld + i] += v) unless its flags mark them shared
// (atomic adds) or staged (stored into its rows of stage, column stride
// sld); outputs are mapped through ymap where its flags say so.  With qjob
// the quadratic forms go to qjob[j * njobs + job] instead of the slots.
template <class T>
void launch_panels(int group, int R, const PanelJob* jobs, const PanelTile* tiles, int njobs,
                   const T* M, const double* xv, int xld, const int* gidx, double* y, int yld,
                   const int* ymap, double* qslot, const int* done, hipStream_t st,
                   double* stage = nullptr, int sld = 0, double* qjob = nullptr);
// Deterministic sums: staged rows into their targets (fixed order per
// target), per-job quadratic forms into slot 0 of each column.
void launch_stage_add(int n, const int* tgt, const int* ptr, const int* idx, const double* stage,
                      int sld, int R, double* y, int yld, const int* done, hipStream_t st);
void launch_qjob_add(int R, int njobs, const double* qjob, double* slots, const int* done,
                     hipStream_t st);
template <class T>
void launch_bdiag(const DevPatch* P, int np, const T* A, double* out, hipStream_t st);
// Tile-path PCG on R (1..4) right-hand sides, column-major vectors; st[R].done
// is the all-columns flag.
void launch_pcg_init_t(int R, int n, const double* d, double* lam, double* r, double* part_dd,
                       int npart, hipStream_t st);
void launch_pcg_init_w(int R, int n, const int* pp, const int* pm, const double* w, int wld,
                       double dt, const double* d, double* r, double* part_dd, int npart,
                       hipStream_t st);
void launch_pcg_init2_t(int R, int n, const int* pp, const int* pm, const double* tb, int tld,
                        const double* wp, const double* wm, const double* rz_slots,
                        const double* part_dd, int npart, PcgScalars* stt, double* p,
                        hipStream_t st);
void launch_pcg_update_t(int R, int n, const int* pp, const int* pm, const double* w, int wld,
                         double dt, const double* pq_slots, PcgScalars* stt, int par,
                         double* lam, double* r, const double* p, double* part_rr, int npart,
                         double* zero, int64_t nzero, hipStream_t st);
void launch_pcg_pupdate_t(int R, int n, const int* pp, const int* pm, const double* tb, int tld,
                          const double* wp, const double* wm, const double* rz_slots,
                          const double* part_rr, int npart, PcgScalars* stt, int par,
                          double tol2, double* p, double* zero, int64_t nzero, hipStream_t st);
// Timing events for the next launch (of a timed kernel) issued by this thread.
void set_launch_events(hipEvent_t start, hipEvent_t stop);
bool launch_events_pending();
void launch_copy_probe(int64_t n32, const void* a, void* b, hipStream_t st);
void launch_read_probe(int64_t n16, const void* a, double* out, hipStream_t st);
// Coarse factor fronts (nested dissection over the patch grid).
template <class T>
void launch_front_add(const DevPatch* P, int s, int n_p, const int* p_nd, const T* A,
                      const CoarseNodeDev* nodes, const int* node_of, const int* slist, double* F,
                      hipStream_t st);
void launch_extend_add(const CoarseNodeDev* nodes, int c, int ns, const int* cpos, double* F,
                       hipStream_t st);
void launch_front_pad(const CoarseNodeDev* nodes, int nn, double* F, hipStream_t st);
void launch_front_rhs(const CoarseNodeDev* nodes, const int* jobs, const int* prefix, int njobs,
                      int total, const double* F, double* L, hipStream_t st);
// dst[j * dld + i] = scale * (w ? w[i] : 1) * src[j * sld + idx[i]], i < n,
// j < R: the gathered (and signed) inputs of the row-panel products, so that
// the panels read them as contiguous blocks.
void launch_gather_cols(int R, int n, const int* idx, const double* w, double scale,
                        const double* src, int sld, double* dst, int dld, const int* done,
                        hipStream_t st);
void launch_sumsq_slots(int R, int n, const double* y, int ld, double* slots, const int* done,
                        hipStream_t st);
void launch_zero(int64_t n, double* a, hipStream_t st);
}  // namespace tcf

// Launchers of the device kernels (kernels_sparse.hip, kernels_dense.hip).
#pragma once

#include "common.h"

namespace nsp {

// sparse
template <typename VT>
void spmm_block(nsp_ctx* c, const Csr& a, int d, const VT* x, VT* y);
// returns the number of per-block Xi partials written to part_xi (the grid size)
template <typename VT>
int spmmT_step(nsp_ctx* c, int d, const VT* y, const VT* x, const VT* xp, const double* gprev,
               VT* out, double* part_xi);
// Y = A X for row-major blocks of k columns; with ``part`` (kWideBlocks x k
// doubles) it also leaves per-block column sums there — of Y^2, or with
// ``dot`` (square A) of Y .* X — and returns the number of blocks for
// reduce_parts.
int spmm_wide(nsp_ctx* c, const Csr& a, int k, const double* x, double* y, double* part = nullptr,
              bool dot = false);
// out[v] = sum_b part[b * nv + v] (fixed order)
void reduce_parts(nsp_ctx* c, int nparts, int nv, const double* part, double* out);
void sddmm(nsp_ctx* c, int k, const double* u, const double* v, double* grad);
void colmajor_to_rows(nsp_ctx* c, int64_t rows, int k, const double* src, int64_t ld, double* dst);
void rows_to_colmajor(nsp_ctx* c, int64_t rows, int k, const double* src, double* dst, int64_t ld);

// arguments of the W-recurrence (Sec. 4.2), evaluated inside the final QR kernel
struct WArgs {
  int ell, l0, ldw;
  double u_d, u_ro;
  const double *n_xi, *n_gam, *n_theta, *n_f;
  double* w;
  int* flags;
  int* hist;  // optional: per-step record of the reorthogonalisation flag
};

// dense: Lanczos step.  Each returns its grid size = number of partials written.
// Xi partials X^T P for block size 8 (n x 8 row-interleaved X and P) on the
// matrix cores; returns the number of partials written to part.
template <typename VT>
int xi8_parts(nsp_ctx* c, int64_t n, const VT* x, const VT* p, double* part);
template <typename VT>
int sub_gram(nsp_ctx* c, int d, int64_t n, VT* p, const VT* x, const double* part_xi, int nparts_xi,
             double* xi_out, double* nrm_xi, double* part_g);
template <typename VT>
int scale_block(nsp_ctx* c, int d, int64_t n, const VT* p, const double* part_g, int nparts,
                VT* xn, VT* zcol, int64_t ldz, double* gam_out, double* nrm_gam, double* nrm_ginv,
                double* part_g2, const WArgs* wa = nullptr);
template <typename VT>
void scale_block2(nsp_ctx* c, int d, int64_t n, const double* part_g2, int nparts, VT* xn, VT* zcol,
                  int64_t ldz, double* gam, double* nrm_gam, double* nrm_ginv,
                  const WArgs* wa = nullptr);
void w_reset(nsp_ctx* c, int col0, int ncols, double u_d, double* w, int ldw);

// dense: tall-skinny projection pair (one CGS pass) and final scaling
int64_t ts_chunk_rows(int64_t n, int k, int nc, int esize = 8);
int64_t ts_part_c_len(int64_t n, int nc);
// FP64 projection h = Z^T C (k x d, basis-column major) and update C -= Z h on
// their own, C row-interleaved n x d (d = 1, 2, 4, 8), Z column-major with an
// even ldz; hpart holds ts_tn_parts_len(n, k, d) doubles
int64_t ts_tn_parts_len(int64_t n, int k, int d);
void ts_tn_only(nsp_ctx* c, int d, int64_t n, const double* z, int64_t ldz, int k, const double* a0,
                double* h, double* hpart);
void ts_nn_only(nsp_ctx* c, int d, int64_t n, const double* z, int64_t ldz, int k, const double* h,
                double* a0);
template <typename VT>
void ts_project(nsp_ctx* c, const int* cond, int d, int na, int64_t n, const VT* z, int64_t ldz,
                int k, VT* a0, VT* a1, double* h, double* hpart, bool gram, double* part_c,
                double* rinv, hipEvent_t ev_tn = nullptr, hipEvent_t ev_red = nullptr);
// C = C R^{-1}; R from the Gram partials of the preceding ts_project(gram) (R^{-1}, R -> rinv)
template <typename VT>
void ts_scale(nsp_ctx* c, const int* cond, int d, int na, int64_t n, VT* a0, VT* a1,
              const double* part_c, double* rinv, VT* z0, int64_t ldz);

// dense: restart / extraction
void assemble_t(nsp_ctx* c, int K, int d, int kk, const double* theta, const double* f,
                const double* xi, const double* gam, double* t);
// F = R Gamma_L V_Z(K-d:K, 0:kn), theta_kept = evals[0:kn], kept-block norms
void restart_coupling(nsp_ctx* c, int K, int d, int kn, const double* vz, const double* gam_l,
                      const double* rinvc, const double* evals, double* f, double* theta_kept,
                      double* n_theta, double* n_f);
template <typename SRC, typename DST>
void cm_to_ri(nsp_ctx* c, int64_t n, int d, const SRC* s, int64_t ld, DST* o);
template <typename SRC, typename DST>
void convert(nsp_ctx* c, int64_t cnt, const SRC* s, DST* o);
template <typename SRC, typename DST>
void copy_panel(nsp_ctx* c, int64_t rows, int cols, const SRC* s, int64_t lds, DST* o, int64_t ldo);

// Ritz eigenproblem of the restart matrix, any block size (eig.hip)
struct EigWork;
EigWork* eig_work_new();
void eig_work_delete(EigWork* w);
void eig_restart(nsp_ctx* c, EigWork& w, int K, int d, int kk, double norm_t, const double* theta,
                 const double* f, const double* xi, const double* gam, double* evals, double* evecs);

// dense: refinement / backward
void coldots(nsp_ctx* c, int64_t rows, int k, const double* a, const double* b, double* out,
             double* part);
int64_t coldots_parts(int64_t rows);
void cgls_xs(nsp_ctx* c, int64_t n, int64_t m, int k, const double* gamma, const double* qq,
             const int* active, double* x, const double* p, double* s, const double* q);
void cgls_p(nsp_ctx* c, int64_t n, int k, const double* gnew, const double* gamma, const int* active,
            const double* r, double* p);
void cg_wr(nsp_ctx* c, int64_t n, int k, const double* rr, const double* pq, const int* active,
           double* w, const double* p, double* r, const double* q);
void sub_inplace(nsp_ctx* c, int64_t cnt, double* x, const double* y);
// x(i, :) /= s[i] (divide) or *= s[i], x row-major rows x k
void scale_rows(nsp_ctx* c, int64_t rows, int k, const double* s, bool divide, double* x);

}  // namespace nsp

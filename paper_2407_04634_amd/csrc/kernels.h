// Launchers of the device kernels (kernels_sparse.hip, kernels_dense.hip).
#pragma once

#include "common.h"

namespace nsp {

// sparse
template <typename VT>
void spmm_block(nsp_ctx* c, const Csr& a, int d, const VT* x, VT* y);
template <typename VT>
void spmmT_step(nsp_ctx* c, int d, const VT* y, const VT* x, const VT* xp, const double* gprev,
                VT* out, double* xi_out, double* xi_nrm = nullptr);
void spmm_wide(nsp_ctx* c, const Csr& a, int k, const double* x, double* y);
void sddmm(nsp_ctx* c, int k, const double* u, const double* v, double* grad);
void colmajor_to_rows(nsp_ctx* c, int64_t rows, int k, const double* src, int64_t ld, double* dst);
void rows_to_colmajor(nsp_ctx* c, int64_t rows, int k, const double* src, double* dst, int64_t ld);

// dense: Lanczos step
template <typename VT>
void sub_gram(nsp_ctx* c, int d, int64_t n, VT* p, const VT* x, const double* xi, double* gam_out,
              double* rinv, double* nrm_gam, double* nrm_ginv);
template <typename VT>
void scale_block(nsp_ctx* c, int d, int64_t n, const VT* p, const double* rinv, VT* xn, VT* zcol,
                 int64_t ldz, bool gram, double* gam, double* rinv2, double* nrm_gam,
                 double* nrm_ginv);
void wrec(nsp_ctx* c, int ell, int l0, double u_d, double u_ro, const double* n_xi,
          const double* n_gam, const double* n_ginv, const double* n_theta, const double* n_f,
          double* w, int ldw);
void w_reset(nsp_ctx* c, int col0, int ncols, double u_d, double* w, int ldw);

// dense: tall-skinny projection pair (CGS pass) and final scaling
int64_t ts_chunk_rows(int64_t n, int k, int nc);
template <typename VT>
void ts_project(nsp_ctx* c, const int* cond, int d, int na, int64_t n, const VT* z, int64_t ldz,
                int k, VT* a0, VT* a1, double* h, double* hpart, bool gram, double* rinv);
template <typename VT>
void ts_scale(nsp_ctx* c, const int* cond, int d, int na, int64_t n, VT* a0, VT* a1,
              const double* rinv, VT* z0, int64_t ldz);

// dense: restart / extraction
void assemble_t(nsp_ctx* c, int K, int d, int kk, const double* theta, const double* f,
                const double* xi, const double* gam, double* t);
template <typename SRC, typename DST>
void cm_to_ri(nsp_ctx* c, int64_t n, int d, const SRC* s, int64_t ld, DST* o);
template <typename SRC, typename DST>
void convert(nsp_ctx* c, int64_t cnt, const SRC* s, DST* o);
template <typename SRC, typename DST>
void copy_panel(nsp_ctx* c, int64_t rows, int cols, const SRC* s, int64_t lds, DST* o, int64_t ldo);

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

}  // namespace nsp

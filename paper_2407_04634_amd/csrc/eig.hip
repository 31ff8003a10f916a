// Eigen-decomposition of the restart matrix T (Eq. "defT") for block size 1.
//
// After a thick restart T = [diag(theta) f 0; f^T a1 b1 ...; 0 tridiagonal tail]:
// kk kept Ritz values theta (ascending) bordered by the coupling row f, the
// arrow tip a1 = Xi_{l0+1}, and a tridiagonal tail.  Cuppen's tear at the
// coupling b1 = Gamma_{l0+1} between the tip and the tail writes
//     T = diag(M1 - b1 e_tip e_tip^T, T2 - b1 e_0 e_0^T) + b1 v v^T,
// v = e_tip + e_{kk+1}.  M1 is an arrowhead ("bordered diagonal") matrix whose
// eigenvalues are the roots of the secular equation
//     a - l - sum_i f_i^2 / (theta_i - l) = 0,
// the tail is tridiagonal (rocSOLVER's divide and conquer), and the rank-one
// merge solves 1 + b1 sum_i z_i^2 / (d_i - l) = 0.  Both secular problems use
// deflation of negligible couplings and of (nearly) equal poles by Givens
// rotations, roots found by bisection on a shifted variable (l = pole + tau,
// so differences l - pole keep full relative accuracy), and Loewner-formula
// weights (Gu & Eisenstat) so that the computed eigenvectors are orthogonal to
// working precision.  The first cycle (no kept vectors) has a plain
// tridiagonal T and goes to the tridiagonal solver directly.
#include <algorithm>
#include <cmath>

#include "common.h"
#include "kernels.h"

namespace nsp {

namespace {

constexpr double kU = 1.1102230246251565e-16;  // 2^-53, rounding unit for the deflation tolerance

inline unsigned nb(int64_t work, int per) { return (unsigned)((work + per - 1) / per); }

// Secular problem descriptor (device arrays, counts on the device).
struct Sec {
  int* cnt;       // [0] n' non-deflated poles, [1] number of rotations, [2] number deflated
  double* p;      // poles (ascending, distinct), n'
  double* w;      // weights (f^2 or z^2), n'
  int* idx;       // row index of each pole in the problem's index space, n'
  int* rot_i;     // rotations (i, j, c, s) in recording order
  int* rot_j;
  double* rot_c;
  double* rot_s;
  double* dval;   // deflated eigenvalues (ascending by recording order of indices)
  int* didx;      // their row index
  int* ro;        // root origin pole index
  double* rt;     // root shift tau
  double* what;   // Loewner weights (signed square roots)
};

// -------------------------------------------------------------------------
// deflation (one thread; sequential over the sorted poles)
//   ARROW: rows 0..m-2 are the poles (value val[i], coupling cpl[i]),
//          row m-1 is the arrow tip; weight = cpl^2.
//   RANK1: rows 0..m-1 are the poles (val[i] sorted ascending), coupling
//          cpl[i]; weight = cpl^2 (rho applied in the root finder).
// -------------------------------------------------------------------------
__global__ void k_deflate(int npoles, const double* __restrict__ val, const double* __restrict__ cpl,
                          const double* cscale_ptr, double scale, Sec s) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double tol = 8.0 * kU * scale;
  // a coupling is negligible when its contribution (times rho for the merge) is below tol
  const double cscale = cscale_ptr ? fabs(*cscale_ptr) : 1.0;
  int np = 0, nr = 0, nd = 0;
  int last = -1;         // row index of the last kept pole
  double last_f = 0.0;   // its (rotated) coupling
  double last_v = 0.0;
  for (int i = 0; i < npoles; ++i) {
    const double v = val[i];
    double fi = cpl[i];
    if (fabs(fi) * cscale <= tol) {
      s.dval[nd] = v;
      s.didx[nd++] = i;
      continue;
    }
    if (last >= 0 && v - last_v <= tol) {
      // rotate (last, i) so that the coupling of ``last`` vanishes; ``last`` deflates
      const double r = hypot(last_f, fi);
      const double c = fi / r, sn = last_f / r;
      s.rot_i[nr] = last;
      s.rot_j[nr] = i;
      s.rot_c[nr] = c;
      s.rot_s[nr++] = sn;
      s.dval[nd] = last_v;
      s.didx[nd++] = last;
      --np;  // drop ``last`` from the kept poles
      fi = r;
    }
    s.p[np] = v;
    s.w[np] = fi * fi;
    s.idx[np] = i;
    // the coupling sign is needed for the eigenvector signs: keep it in what
    s.what[np] = fi;
    ++np;
    last = i;
    last_f = fi;
    last_v = v;
  }
  s.cnt[0] = np;
  s.cnt[1] = nr;
  s.cnt[2] = nd;
}

// secular functions in the shifted variable tau (lambda = p[o] + tau); one
// wavefront evaluates the sum, every lane returns the same value
__device__ __forceinline__ double wave_sum64(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <bool ARROW>
__device__ double sec_eval(int np, const double* p, const double* w, int o, double tau, double a_or_rho) {
  const double po = p[o];
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += 64) s += w[i] / ((p[i] - po) - tau);
  s = wave_sum64(s);
  if (ARROW) return (a_or_rho - po) - tau - s;  // decreasing in tau
  return 1.0 + a_or_rho * s;                    // increasing in tau (rho > 0)
}

// roots: ARROW has n'+1 roots (one below p0, one per gap, one above), RANK1 has
// n'; one 64-lane block per root
template <bool ARROW>
__global__ __launch_bounds__(64) void k_roots(Sec s, const double* a_or_rho_ptr, double lo_bound,
                                              double hi_bound) {
  const int np = s.cnt[0];
  const int nroots = ARROW ? np + 1 : np;
  const int j = blockIdx.x;
  if (j >= nroots) return;
  const double ar = *a_or_rho_ptr;
  if (ARROW && np == 0) {  // every coupling deflated: the tip is an eigenvalue
    if (threadIdx.x == 0) {
      s.ro[0] = -1;
      s.rt[0] = ar;
    }
    return;
  }
  const double* p = s.p;
  const double* w = s.w;
  int o;
  double lo, hi;
  if (ARROW) {
    if (j == 0) {
      o = 0; lo = lo_bound - p[0]; hi = 0.0;
    } else if (j == np) {
      o = np - 1; lo = 0.0; hi = hi_bound - p[np - 1];
    } else {
      const double h = p[j] - p[j - 1];
      const double gm = sec_eval<true>(np, p, w, j - 1, 0.5 * h, ar);
      if (gm > 0.0) { o = j; lo = -0.5 * h; hi = 0.0; }       // root in the right half
      else { o = j - 1; lo = 0.0; hi = 0.5 * h; }
    }
  } else {
    if (j == np - 1) {
      double sw = 0.0;
      for (int i = threadIdx.x; i < np; i += 64) sw += w[i];
      sw = wave_sum64(sw);
      o = np - 1; lo = 0.0; hi = ar * sw;
    } else {
      const double h = p[j + 1] - p[j];
      const double fm = sec_eval<false>(np, p, w, j, 0.5 * h, ar);
      if (fm > 0.0) { o = j; lo = 0.0; hi = 0.5 * h; }         // root in the left half
      else { o = j + 1; lo = -0.5 * h; hi = 0.0; }
    }
  }
  // bisection to floating-point resolution (all lanes take the same branches)
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    const double g = sec_eval<ARROW>(np, p, w, o, mid, ar);
    const bool right = ARROW ? (g > 0.0) : (g < 0.0);
    if (right) lo = mid; else hi = mid;
  }
  if (threadIdx.x == 0) {
    s.ro[j] = o;
    s.rt[j] = 0.5 * (lo + hi);
  }
}

// lambda_k - p_i with full accuracy
__device__ __forceinline__ double lam_minus(const Sec& s, int k, int i) {
  return (s.p[s.ro[k]] - s.p[i]) + s.rt[k];
}

__device__ __forceinline__ double root_val(const Sec& s, int k) {
  return s.ro[k] < 0 ? s.rt[k] : s.p[s.ro[k]] + s.rt[k];
}

// Loewner weights: signed square roots of the weights for which the computed
// roots are exact eigenvalues (pairing the factors keeps every ratio bounded).
template <bool ARROW>
__global__ void k_lowner(Sec s, const double* a_or_rho_ptr) {
  const int np = s.cnt[0];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  const double* p = s.p;
  double prod;
  if (ARROW) {
    // f_i^2 = -(p_i - l_i)(p_i - l_{i+1}) prod_{k<i} (p_i - l_k)/(p_i - p_k)
    //                                      prod_{k>i} (p_i - l_{k+1})/(p_i - p_k)
    prod = lam_minus(s, i, i) * lam_minus(s, i + 1, i);  // (l_i - p_i)(l_{i+1} - p_i) < 0
    prod = -prod;
    for (int k = 0; k < i; ++k) prod *= (-lam_minus(s, k, i)) / (p[i] - p[k]);
    for (int k = i + 1; k < np; ++k) prod *= (-lam_minus(s, k + 1, i)) / (p[i] - p[k]);
  } else {
    // z_i^2 = -(1/rho)(d_i - l_{n-1}) prod_{k<i} (d_i - l_k)/(d_i - d_k)
    //                                 prod_{k>i} (d_i - l_{k-1})/(d_i - d_k)
    const double rho = *a_or_rho_ptr;
    prod = lam_minus(s, np - 1, i) / rho;  // (l_{n-1} - d_i)/rho > 0
    for (int k = 0; k < i; ++k) prod *= (-lam_minus(s, k, i)) / (p[i] - p[k]);
    for (int k = i + 1; k < np; ++k) prod *= (-lam_minus(s, k - 1, i)) / (p[i] - p[k]);
  }
  const double sign = s.what[i] < 0.0 ? -1.0 : 1.0;
  s.what[i] = sign * sqrt(fmax(prod, 0.0));
}

// Eigenvector of root j (one block per root), written as column j of X
// (ldx rows, row index space of the problem).  ARROW: entries at the pole
// rows and 1 at the tip row; RANK1: entries at the pole rows.
template <bool ARROW>
__global__ void k_vectors(Sec s, double* x, int ldx, int tip_row) {
  const int np = s.cnt[0];
  const int nroots = ARROW ? np + 1 : np;
  const int j = blockIdx.x;
  if (j >= nroots) return;
  __shared__ double red[256];
  double ss = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) {
    const double den = ARROW ? lam_minus(s, j, i) : -lam_minus(s, j, i);  // l_j - p_i  |  d_i - l_j
    const double v = s.what[i] / den;
    ss += v * v;
  }
  red[threadIdx.x] = ss;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  const double nrm = sqrt(red[0] + (ARROW ? 1.0 : 0.0));
  double* col = x + (int64_t)j * ldx;
  for (int i = threadIdx.x; i < np; i += blockDim.x) {
    const double den = ARROW ? lam_minus(s, j, i) : -lam_minus(s, j, i);
    col[s.idx[i]] = s.what[i] / den / nrm;
  }
  if (ARROW && threadIdx.x == 0) col[tip_row] = 1.0 / nrm;
}

// deflated columns: unit vectors at their rows, in the last nd of the m
// columns (the secular roots fill the first m - nd)
__global__ void k_deflated_cols(Sec s, double* x, int ldx, int m) {
  const int nd = s.cnt[2];
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nd) return;
  x[(int64_t)(m - nd + q) * ldx + s.didx[q]] = 1.0;
}

// undo the deflation rotations on the rows of X (latest first), all columns
__global__ void k_unrotate(Sec s, double* x, int ldx, int ncols) {
  const int nr = s.cnt[1];
  for (int r = nr - 1; r >= 0; --r) {
    const int pi = s.rot_i[r], pj = s.rot_j[r];
    const double c = s.rot_c[r], sn = s.rot_s[r];
    for (int col = threadIdx.x; col < ncols; col += blockDim.x) {
      double* xc = x + (int64_t)col * ldx;
      const double a = xc[pi], b = xc[pj];
      xc[pi] = c * a + sn * b;
      xc[pj] = -sn * a + c * b;
    }
    __syncthreads();
  }
}

// ascending (value, column) list from the secular roots (columns 0..nroots-1)
// and the deflated values (columns nroots..), merging two sorted sequences;
// the deflated values are first sorted by insertion (few, nearly sorted)
template <bool ARROW>
__global__ void k_order(Sec s, double* lam, int* col) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int np = s.cnt[0], nd = s.cnt[2];
  const int nroots = ARROW ? np + 1 : np;
  // insertion sort of the deflated list (stable, by value) carrying the index
  for (int a = 1; a < nd; ++a) {
    const double v = s.dval[a];
    const int id = s.didx[a];
    int b = a - 1;
    while (b >= 0 && s.dval[b] > v) {
      s.dval[b + 1] = s.dval[b];
      s.didx[b + 1] = s.didx[b];
      --b;
    }
    s.dval[b + 1] = v;
    s.didx[b + 1] = id;
  }
  int r = 0, q = 0, k = 0;
  while (r < nroots || q < nd) {
    const double lr = r < nroots ? root_val(s, r) : INFINITY;
    const double lq = q < nd ? s.dval[q] : INFINITY;
    if (lr <= lq) { lam[k] = lr; col[k++] = r++; }
    else { lam[k] = lq; col[k++] = nroots + q++; }
  }
}

// tail tridiagonal (d = 1): diag a_{l0+2..L} (first reduced by b), offdiag b_{l0+2..L-1}
__global__ void k_tail(int m2, const double* __restrict__ xi, const double* __restrict__ gam,
                       int first_blk, double* __restrict__ dd, double* __restrict__ ee) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m2) return;
  const double b = gam[first_blk - 1];  // Gamma_{l0+1}: coupling to the arrow tip
  dd[i] = xi[first_blk + i] - (i == 0 ? b : 0.0);
  if (i + 1 < m2) ee[i] = gam[first_blk + i];
}

// full tridiagonal (first cycle): diag a_1..a_L, offdiag b_1..b_{L-1}
__global__ void k_tridiag(int L, const double* __restrict__ xi, const double* __restrict__ gam,
                          double* __restrict__ dd, double* __restrict__ ee) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= L) return;
  dd[i] = xi[1 + i];
  if (i + 1 < L) ee[i] = gam[1 + i];
}

// arrow data: poles theta (kk), couplings f (kk), tip a1 - b1, scale
__global__ void k_arrow_tip(const double* __restrict__ xi, const double* __restrict__ gam, int blk,
                            double* tip) {
  if (threadIdx.x == 0 && blockIdx.x == 0) tip[0] = xi[blk] - gam[blk];  // a1 - b1
}

// the merge problem: union of the arrow eigenvalues (lam1/col1 over U1) and the
// tail eigenvalues (ascending, columns of U2); couplings z = U1[tip, col] and
// U2[0, col]; src[k] = column in U1 (>= 0) or -(1 + column in U2)
__global__ void k_merge_union(int m1, int m2, const double* __restrict__ lam1,
                              const int* __restrict__ col1, const double* __restrict__ u1,
                              const double* __restrict__ lam2, const double* __restrict__ u2,
                              double* __restrict__ d, double* __restrict__ z, int* __restrict__ src) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int a = 0, b = 0, k = 0;
  while (a < m1 || b < m2) {
    const double va = a < m1 ? lam1[a] : INFINITY;
    const double vb = b < m2 ? lam2[b] : INFINITY;
    if (va <= vb) {
      d[k] = va;
      z[k] = u1[(int64_t)col1[a] * m1 + (m1 - 1)];
      src[k++] = col1[a++];
    } else {
      d[k] = vb;
      z[k] = u2[(int64_t)b * m2];
      src[k++] = -(1 + b++);
    }
  }
}

// scatter the merge eigenvectors (rows = union index, natural column order) to
// Wa (m1 x K, rows = U1 columns) and Wt (m2 x K, rows = U2 columns), columns in
// final ascending order
__global__ void k_scatter(int K, int m1, int m2, const double* __restrict__ wn,
                          const int* __restrict__ src, const int* __restrict__ colf,
                          double* __restrict__ wa, double* __restrict__ wt) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)K * K) return;
  const int k = (int)(e % K), j = (int)(e / K);  // union row k, final column j
  const double v = wn[(int64_t)colf[j] * K + k];
  const int sc = src[k];
  if (sc >= 0) wa[(int64_t)j * m1 + sc] = v;
  else wt[(int64_t)j * m2 + (-sc - 1)] = v;
}

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct EigWork {
  DBuf b_int, b_dbl, b_u1, b_u2, b_wn, b_wa, b_wt, b_dd, b_ee, b_info;
};

static Sec make_sec(double*& dp, int*& ip, int m) {
  Sec s;
  s.cnt = ip; ip += 4;
  s.p = dp; dp += m;
  s.w = dp; dp += m;
  s.idx = ip; ip += m;
  s.rot_i = ip; ip += m;
  s.rot_j = ip; ip += m;
  s.rot_c = dp; dp += m;
  s.rot_s = dp; dp += m;
  s.dval = dp; dp += m;
  s.didx = ip; ip += m;
  s.ro = ip; ip += m + 1;
  s.rt = dp; dp += m + 1;
  s.what = dp; dp += m;
  return s;
}

static void stedc(nsp_ctx* c, int n, double* dd, double* ee, double* cvec, rocblas_int* info) {
  NSP_BLAS(rocsolver_dstedc(c->blas, rocblas_evect_tridiagonal, n, dd, ee, cvec, n, info));
}

// Eigen-decomposition of T for d = 1 (see the file comment).  xi and gam are
// indexed by Lanczos block number (xi[j] = Xi_j, gam[j] = Gamma_j); theta and
// f hold the kk kept Ritz values and couplings.  norm_t bounds ||T||.  On
// return evecs (K x K, column-major) holds the eigenvectors and evals the
// eigenvalues, ascending; *info_dev receives the tridiagonal solver's info.
void eig_restart_d1(nsp_ctx* c, EigWork& w, int K, int kk, double norm_t, const double* theta,
                    const double* f, const double* xi, const double* gam, double* evals,
                    double* evecs, int* info_dev) {
  rocblas_int* info = reinterpret_cast<rocblas_int*>(info_dev);
  if (kk == 0) {
    w.b_ee.alloc(sizeof(double) * (size_t)K);
    k_tridiag<<<nb(K, 256), 256, 0, c->stream>>>(K, xi, gam, evals, w.b_ee.as<double>());
    NSP_HIP(hipGetLastError());
    stedc(c, K, evals, w.b_ee.as<double>(), evecs, info);
    return;
  }
  const int l0 = kk;  // d = 1: kept blocks = kept vectors
  const int m1 = kk + 1, m2 = K - kk - 1;
  w.b_int.alloc(sizeof(int) * (size_t)(24 * (K + 8)));
  w.b_dbl.alloc(sizeof(double) * (size_t)(24 * (K + 8)));
  w.b_u1.alloc(sizeof(double) * (size_t)m1 * m1);
  w.b_u2.alloc(sizeof(double) * (size_t)m2 * m2);
  w.b_wn.alloc(sizeof(double) * (size_t)K * K);
  w.b_wa.alloc(sizeof(double) * (size_t)m1 * K);
  w.b_wt.alloc(sizeof(double) * (size_t)m2 * K);
  w.b_dd.alloc(sizeof(double) * (size_t)(m2 + 8));
  w.b_ee.alloc(sizeof(double) * (size_t)(m2 + 8));
  double* dp = w.b_dbl.as<double>();
  int* ip = w.b_int.as<int>();
  Sec sa = make_sec(dp, ip, m1);
  Sec sm = make_sec(dp, ip, K);
  double* tip = dp; dp += 2;
  double* lam1 = dp; dp += m1;
  double* lam = dp; dp += K;
  double* dvals = dp; dp += K;
  double* zc = dp; dp += K;
  int* col1 = ip; ip += m1;
  int* colf = ip; ip += K;
  int* src = ip; ip += K;
  double* u1 = w.b_u1.as<double>();
  double* u2 = w.b_u2.as<double>();
  double* wn = w.b_wn.as<double>();
  double* dd = w.b_dd.as<double>();
  double* ee = w.b_ee.as<double>();
  const double bound = 4.0 * norm_t + 1.0;  // every eigenvalue of the arrowhead lies inside

  // ---- arrowhead M1 = [diag(theta) f; f^T Xi_{l0+1} - Gamma_{l0+1}]
  k_arrow_tip<<<1, 1, 0, c->stream>>>(xi, gam, l0 + 1, tip);
  k_deflate<<<1, 1, 0, c->stream>>>(kk, theta, f, nullptr, norm_t, sa);
  k_roots<true><<<m1, 64, 0, c->stream>>>(sa, tip, -bound, bound);
  k_lowner<true><<<nb(m1, 128), 128, 0, c->stream>>>(sa, tip);
  NSP_HIP(hipMemsetAsync(u1, 0, sizeof(double) * (size_t)m1 * m1, c->stream));
  k_vectors<true><<<m1, 256, 0, c->stream>>>(sa, u1, m1, m1 - 1);
  k_order<true><<<1, 1, 0, c->stream>>>(sa, lam1, col1);
  k_deflated_cols<<<nb(m1, 256), 256, 0, c->stream>>>(sa, u1, m1, m1);
  k_unrotate<<<1, 1024, 0, c->stream>>>(sa, u1, m1, m1);
  NSP_HIP(hipGetLastError());

  // ---- tail T2 - Gamma_{l0+1} e_0 e_0^T (tridiagonal)
  k_tail<<<nb(m2, 256), 256, 0, c->stream>>>(m2, xi, gam, l0 + 2, dd, ee);
  NSP_HIP(hipGetLastError());
  stedc(c, m2, dd, ee, u2, info);

  // ---- rank-one merge with rho = Gamma_{l0+1}
  const double* rho = gam + (l0 + 1);
  k_merge_union<<<1, 1, 0, c->stream>>>(m1, m2, lam1, col1, u1, dd, u2, dvals, zc, src);
  k_deflate<<<1, 1, 0, c->stream>>>(K, dvals, zc, rho, norm_t, sm);
  k_roots<false><<<K, 64, 0, c->stream>>>(sm, rho, 0.0, 0.0);
  k_lowner<false><<<nb(K, 128), 128, 0, c->stream>>>(sm, rho);
  NSP_HIP(hipMemsetAsync(wn, 0, sizeof(double) * (size_t)K * K, c->stream));
  k_vectors<false><<<K, 256, 0, c->stream>>>(sm, wn, K, 0);
  k_order<false><<<1, 1, 0, c->stream>>>(sm, lam, colf);
  k_deflated_cols<<<nb(K, 256), 256, 0, c->stream>>>(sm, wn, K, K);
  k_unrotate<<<1, 1024, 0, c->stream>>>(sm, wn, K, K);
  NSP_HIP(hipGetLastError());

  // ---- eigenvectors of T = [U1 0; 0 U2] W, columns ascending
  k_scatter<<<nb((int64_t)K * K, 256), 256, 0, c->stream>>>(K, m1, m2, wn, src, colf,
                                                            w.b_wa.as<double>(), w.b_wt.as<double>());
  NSP_HIP(hipGetLastError());
  const double one = 1.0, zero = 0.0;
  NSP_BLAS(rocblas_dgemm(c->blas, rocblas_operation_none, rocblas_operation_none, m1, K, m1, &one, u1,
                         m1, w.b_wa.as<double>(), m1, &zero, evecs, K));
  NSP_BLAS(rocblas_dgemm(c->blas, rocblas_operation_none, rocblas_operation_none, m2, K, m2, &one, u2,
                         m2, w.b_wt.as<double>(), m2, &zero, evecs + m1, K));
  NSP_HIP(hipMemcpyAsync(evals, lam, sizeof(double) * K, hipMemcpyDeviceToDevice, c->stream));
}

EigWork* eig_work_new() { return new EigWork(); }
void eig_work_delete(EigWork* w) { delete w; }

}  // namespace nsp

// Eigen-decomposition of the restart matrix T (Eq. "defT") for block size d.
//
// After a thick restart
//     T = [diag(theta)  F^T   0            ]   kk kept Ritz values theta
//         [F            Xi_1  Gamma_1^T    ]   (ascending), their coupling F
//         [0            Gamma_1  Xi_2  ... ]   (d x kk) to the first new block,
//                                              then the block tridiagonal tail
// (Xi_j symmetric d x d on the diagonal, Gamma_j upper triangular below it);
// the first cycle (kk = 0) has the block tridiagonal part only.  Divide and
// conquer in the manner of Cuppen, for d x d blocks:
//  * a coupling Gamma = P S Q^T (SVD) between consecutive blocks is torn:
//        [0 Gamma^T; Gamma 0] = sum_i s_i v_i v_i^T - diag(Q S Q^T, P S P^T),
//    v_i = [q_i; p_i], so the upper block loses Q S Q^T, the lower one
//    P S P^T, and the two halves are joined again by d rank-one updates;
//  * the tail is torn down to its d x d blocks (Jacobi), padded to a power of
//    two with decoupled blocks above every eigenvalue of T, and merged level
//    by level, all merges of a level in one batch;
//  * the kept part with its d-row border is a block arrowhead, solved as d
//    successive arrowheads [diag(lambda) z; z^T x] (one secular equation
//    each, z the next border row in the current eigenbasis);
//  * arrowhead and tail are joined by the d rank-one updates of the tear at
//    the coupling between them.
// Every secular problem uses deflation of negligible couplings and of
// (nearly) equal poles by Givens rotations, roots found by bisection in a
// shifted variable (lambda = pole + tau, so differences lambda - pole keep
// full relative accuracy), and Loewner-formula weights (Gu & Eisenstat) so
// that the computed eigenvectors are orthogonal to working precision.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"
#include "kernels.h"

namespace nsp {

namespace {

constexpr double kU = 1.1102230246251565e-16;  // 2^-53, rounding unit for the deflation tolerance
constexpr int kLdsBytes = 64 * 1024;            // dynamic LDS the secular kernels may stage into

inline unsigned nb(int64_t work, int per) { return (unsigned)((work + per - 1) / per); }

// Secular problem descriptor (device arrays, counts on the device).  A batch of
// problems shares one descriptor: problem b uses every array at offset b * S
// (the counts at offset 4 b).
struct Sec {
  int* cnt;       // [0] n' non-deflated poles, [1] number of rotations, [2] number deflated
  double* p;      // poles (ascending, distinct), n'
  double* w;      // weights (f^2 or z^2), n'
  int* idx;       // row index of each pole in the problem's index space, n'
  int* rot_i;     // rotations (i, j, c, s) in recording order
  int* rot_j;
  double* rot_c;
  double* rot_s;
  double* dval;   // deflated eigenvalues
  int* didx;      // their row index
  int* ro;        // root origin pole index
  double* rt;     // root shift tau
  double* what;   // Loewner weights (signed square roots)
};

__device__ __forceinline__ Sec sec_at(const Sec& s, int b, int S) {
  const int64_t o = (int64_t)b * S;
  Sec r;
  r.cnt = s.cnt + 4 * b;
  r.p = s.p + o;
  r.w = s.w + o;
  r.idx = s.idx + o;
  r.rot_i = s.rot_i + o;
  r.rot_j = s.rot_j + o;
  r.rot_c = s.rot_c + o;
  r.rot_s = s.rot_s + o;
  r.dval = s.dval + o;
  r.didx = s.didx + o;
  r.ro = s.ro + o;
  r.rt = s.rt + o;
  r.what = s.what + o;
  return r;
}

// block-wide exclusive scan of one int per thread (Hillis-Steele in LDS);
// *total receives the block's sum in every thread
__device__ int block_excl_scan(int v, int* scratch, int* total) {
  const int t = threadIdx.x;
  scratch[t] = v;
  __syncthreads();
  for (int off = 1; off < (int)blockDim.x; off <<= 1) {
    const int add = t >= off ? scratch[t - off] : 0;
    __syncthreads();
    scratch[t] += add;
    __syncthreads();
  }
  const int incl = scratch[t];
  *total = scratch[blockDim.x - 1];
  __syncthreads();
  return incl - v;
}

// -------------------------------------------------------------------------
// deflation, one block of kDeflThreads per problem
//   ARROW: rows 0..m-1 are the poles (value val[i], coupling cpl[i]); the
//          arrow tip is row m; weight = cpl^2.
//   RANK1: rows 0..m-1 are the poles (val[i] sorted ascending), coupling
//          cpl[i]; weight = cpl^2 (rho applied in the root finder).
// val of problem b at val + b vstride; coupling i at cpl[b cstride + i cinc].
// A coupling is negligible when |cpl| (times |rho| for a merge) <= tol; of the
// others, consecutive poles closer than tol form runs, and a Givens rotation
// moves the coupling of each run member onto the next one, so that all but
// the last of a run deflate and the last carries the run's combined coupling.
// Kept poles and deflated values come out in index (= value) order, the
// rotations run by run in the order they must be undone in reverse.
// -------------------------------------------------------------------------
constexpr int kDeflThreads = 256;

__global__ __launch_bounds__(kDeflThreads) void k_deflate(int npoles, const double* __restrict__ val,
                                                          int64_t vstride, const double* __restrict__ cpl,
                                                          int cinc, int64_t cstride,
                                                          const double* __restrict__ rho, double scale, Sec s0,
                                                          int S) {
  extern __shared__ int shi[];
  int* aidx = shi;                  // non-negligible pole indices (compacted), npoles
  int* cpos = shi + npoles;         // close pairs before A position k, npoles
  unsigned char* dfl = reinterpret_cast<unsigned char*>(shi + 2 * npoles);  // deflated flag per index
  __shared__ int scan[kDeflThreads];
  const int b = blockIdx.x;
  const int t = threadIdx.x, nt = blockDim.x;
  const Sec s = sec_at(s0, b, S);
  const double* v = val + (int64_t)b * vstride;
  const double* cp = cpl + (int64_t)b * cstride;
  const double tol = 8.0 * kU * scale;
  const double cscale = rho ? fabs(rho[b]) : 1.0;
  auto f_of = [&](int i) { return cp[(int64_t)i * cinc]; };
  // pass 1: negligible couplings; compaction of the others into aidx
  const int ch = (npoles + nt - 1) / nt, i0 = min(npoles, t * ch), i1 = min(npoles, i0 + ch);
  int cnt = 0;
  for (int i = i0; i < i1; ++i) {
    const bool neg = fabs(f_of(i)) * cscale <= tol;
    dfl[i] = neg ? 1 : 0;
    cnt += neg ? 0 : 1;
  }
  int na;
  int base = block_excl_scan(cnt, scan, &na);
  for (int i = i0; i < i1; ++i)
    if (!dfl[i]) aidx[base++] = i;
  __syncthreads();
  // pass 2: close pairs (k, k+1) of consecutive kept candidates
  const int kc = (na + nt - 1) / nt, k0 = min(na, t * kc), k1 = min(na, k0 + kc);
  auto close_at = [&](int k) { return k + 1 < na && v[aidx[k + 1]] - v[aidx[k]] <= tol; };
  int ncl = 0;
  for (int k = k0; k < k1; ++k) ncl += close_at(k) ? 1 : 0;
  int nclose;
  int cb = block_excl_scan(ncl, scan, &nclose);
  for (int k = k0; k < k1; ++k) {
    cpos[k] = cb;
    if (close_at(k)) {
      ++cb;
      dfl[aidx[k]] = 1;
    }
  }
  __syncthreads();
  // kept poles (singletons here, run ends by their run's first member) and rotations
  for (int k = k0; k < k1; ++k) {
    const bool cl = close_at(k);
    const bool prev_cl = k > 0 && close_at(k - 1);
    if (!cl && !prev_cl) {
      const int i = aidx[k], kp = k - cpos[k];
      const double fi = f_of(i);
      s.p[kp] = v[i];
      s.w[kp] = fi * fi;
      s.idx[kp] = i;
      s.what[kp] = fi;  // the coupling sign is needed for the eigenvector signs
    } else if (cl && !prev_cl) {
      double last_f = f_of(aidx[k]);
      int q = k;
      while (close_at(q)) {
        const double fn = f_of(aidx[q + 1]);
        const double r = hypot(last_f, fn);
        const int ri = cpos[q];
        s.rot_i[ri] = aidx[q];
        s.rot_j[ri] = aidx[q + 1];
        s.rot_c[ri] = fn / r;
        s.rot_s[ri] = last_f / r;
        last_f = r;
        ++q;
      }
      const int i = aidx[q], kp = q - cpos[q];
      s.p[kp] = v[i];
      s.w[kp] = last_f * last_f;
      s.idx[kp] = i;
      s.what[kp] = last_f;
    }
  }
  // pass 3: deflated values in index order
  int nd0 = 0;
  for (int i = i0; i < i1; ++i) nd0 += dfl[i];
  int nd;
  int db = block_excl_scan(nd0, scan, &nd);
  for (int i = i0; i < i1; ++i)
    if (dfl[i]) {
      s.dval[db] = v[i];
      s.didx[db++] = i;
    }
  if (t == 0) {
    s.cnt[0] = na - nclose;
    s.cnt[1] = nclose;
    s.cnt[2] = nd;
  }
}

// Sum over a wavefront, returned in every lane, with DPP lane moves (a few
// cycles each) instead of LDS permutes: within each row of 16 lanes an
// inclusive scan by row shifts 1, 2, 4, 8; then the row broadcasts of lanes 15
// and 31 carry the row totals up, so lane 63 holds the wavefront's sum, which
// readlane broadcasts.  The wavefront must be converged.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROW_MASK, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double wave_sum64(double v) {
  v += dpp_move<0x111, 0xF>(v);  // row_shr:1
  v += dpp_move<0x112, 0xF>(v);  // row_shr:2
  v += dpp_move<0x114, 0xF>(v);  // row_shr:4
  v += dpp_move<0x118, 0xF>(v);  // row_shr:8
  v += dpp_move<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_move<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// secular functions in the shifted variable tau (lambda = p[o] + tau); one
// wavefront evaluates the sum, every lane returns the same value

template <bool ARROW>
__device__ double sec_eval(int np, const double* p, const double* w, int o, double tau, double a_or_rho,
                           int lane) {
  const double po = p[o];
  double s = 0.0;
  for (int i = lane; i < np; i += 64) s += w[i] / ((p[i] - po) - tau);
  s = wave_sum64(s);
  if (ARROW) return (a_or_rho - po) - tau - s;  // decreasing in tau
  return 1.0 + a_or_rho * s;                    // increasing in tau (rho > 0)
}

// roots: ARROW has n'+1 roots (one below p0, one per gap, one above), RANK1 has
// n'; one wavefront per root, four per block (grid.y = problem), the poles and
// weights staged in LDS when they fit.  a_or_rho: tip or rho per problem.
template <bool ARROW, bool LDS>
__global__ __launch_bounds__(256) void k_roots(Sec s0, int S, const double* __restrict__ a_or_rho,
                                               double lo_bound, double hi_bound) {
  extern __shared__ double sh[];
  const int b = blockIdx.y;
  const Sec s = sec_at(s0, b, S);
  const int np = s.cnt[0];
  const double* p = s.p;
  const double* w = s.w;
  if (LDS) {
    for (int i = threadIdx.x; i < np; i += blockDim.x) {
      sh[i] = s.p[i];
      sh[np + i] = s.w[i];
    }
    __syncthreads();
    p = sh;
    w = sh + np;
  }
  const int nroots = ARROW ? np + 1 : np;
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= nroots) return;
  const double ar = a_or_rho[b];
  if (ARROW && np == 0) {  // every coupling deflated: the tip is an eigenvalue
    if (lane == 0) {
      s.ro[0] = -1;
      s.rt[0] = ar;
    }
    return;
  }
  int o;
  double lo, hi;
  if (ARROW) {
    if (j == 0) {
      o = 0; lo = lo_bound - p[0]; hi = 0.0;
    } else if (j == np) {
      o = np - 1; lo = 0.0; hi = hi_bound - p[np - 1];
    } else {
      const double h = p[j] - p[j - 1];
      const double gm = sec_eval<true>(np, p, w, j - 1, 0.5 * h, ar, lane);
      if (gm > 0.0) { o = j; lo = -0.5 * h; hi = 0.0; }       // root in the right half
      else { o = j - 1; lo = 0.0; hi = 0.5 * h; }
    }
  } else {
    if (j == np - 1) {
      double sw = 0.0;
      for (int i = lane; i < np; i += 64) sw += w[i];
      sw = wave_sum64(sw);
      o = np - 1; lo = 0.0; hi = ar * sw;
    } else {
      const double h = p[j + 1] - p[j];
      const double fm = sec_eval<false>(np, p, w, j, 0.5 * h, ar, lane);
      if (fm > 0.0) { o = j; lo = 0.0; hi = 0.5 * h; }         // root in the left half
      else { o = j + 1; lo = -0.5 * h; hi = 0.0; }
    }
  }
  // Model steps inside the bracket [lo, hi], which every evaluation shrinks;
  // a step that leaves it is replaced by bisection.  The models are fitted to
  // the value and the derivative at tau, so each is exact when only the poles
  // it keeps (and, for the arrowhead, its linear term) contribute.
  //   Interior root between poles jl and jl+1: the sum is split there into psi
  //   (poles jl and below, all terms of one sign) and phi (the rest, the other
  //   sign), each modelled by its pole plus a constant (the "middle way" of
  //   rational secular solvers); the arrowhead's linear term adds its slope
  //   to the nearer pole's weight.  The step solves a quadratic.
  //   Outermost root (poles on one side only): for the rank-one update the
  //   sum is modelled by pole o plus a constant, c + e / (0 - x); for the
  //   arrowhead by C - x + S / x (pole o and the linear term), a quadratic
  //   again.
  // Plain Newton steps from a far bracket end need dozens of bisections when
  // a weight is tiny and the root sits within rounding distance of its pole.
  // A root is accepted once |g| is below the rounding level of its evaluation
  // or once a step reaches the rounding level of tau.  The level bounds what
  // evaluating g at tau can resolve: each term w/d carries a few roundings
  // (d's relative error is a few units, tau staying within half a gap of the
  // pole), the sum adds its own, and one unit of tau moves g by |tau g'|.
  double tau = 0.5 * (lo + hi);
  const bool outer = ARROW ? (j == 0 || j == np) : (j == np - 1);
  const int jl = ARROW ? j - 1 : j;  // interior: the poles left and right of the root
  const double po = p[o];
  const double dl = outer ? 0.0 : p[jl] - po, dr = outer ? 0.0 : p[jl + 1] - po;
  const double kf = ARROW ? -1.0 : ar;  // model: cm + kf (s1 / (a - x) + s2 / (b - x))
  for (int it = 0; it < 200; ++it) {
    double ps = 0.0, dps = 0.0, ph = 0.0, dph = 0.0;
    for (int i = lane; i < np; i += 64) {
      const double r = 1.0 / ((p[i] - po) - tau);
      const double t = w[i] * r;
      if (i <= jl) { ps += t; dps += t * r; }
      else { ph += t; dph += t * r; }
    }
    ps = wave_sum64(ps);
    dps = wave_sum64(dps);
    ph = wave_sum64(ph);
    dph = wave_sum64(dph);
    // psi's terms are all of one sign and phi's of the other, so |psi| + |phi|
    // is the sum of |w / d| the rounding level needs
    const double sa = fabs(ps) + fabs(ph);
    double g, dg, eg;
    if (ARROW) {
      g = (ar - po) - tau - (ps + ph);  // decreasing in tau
      dg = -1.0 - (dps + dph);
      eg = kU * (fabs(ar - po) + fabs(tau) + 8.0 * sa + 3.0 * fabs(tau * dg));
    } else {
      g = 1.0 + ar * (ps + ph);         // increasing in tau (rho > 0)
      dg = ar * (dps + dph);
      eg = kU * (8.0 * (1.0 + ar * sa) + 3.0 * fabs(tau * dg));
    }
    if (fabs(g) <= eg) {
      lo = hi = tau;
      break;
    }
    if (ARROW ? g > 0.0 : g < 0.0) lo = tau; else hi = tau;
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    double x = NAN;  // the model's step, tau + x its root
    if (!outer) {
      // distances a < 0 < b from tau to the two poles
      const double a = dl - tau, bq = dr - tau;
      double s1 = dps * a * a, s2 = dph * bq * bq;
      if (ARROW) {
        if (o == jl) s1 += a * a; else s2 += bq * bq;
      }
      const double cm = g - kf * (s1 / a + s2 / bq);
      const double qa = cm, qb = -(cm * (a + bq) + kf * (s1 + s2)), qc = cm * a * bq + kf * (s1 * bq + s2 * a);
      const double disc = qb * qb - 4.0 * qa * qc;
      if (disc >= 0.0) {
        const double q = -0.5 * (qb + copysign(sqrt(disc), qb));
        const double x1 = qa != 0.0 ? q / qa : NAN;
        const double x2 = q != 0.0 ? qc / q : NAN;
        x = (x1 > a && x1 < bq) ? x1 : x2;
        if (!(x > a && x < bq)) x = NAN;
      }
    } else if (ARROW) {
      // C - x + S / x = 0 with S = -(g' + 1) tau^2 >= 0; the root on tau's side
      // of the pole (positive for j = np, negative for j = 0), taken from the
      // form without cancellation
      const double sq = -(dg + 1.0) * tau * tau;
      const double cc = g + tau - sq / tau;
      const double rt = sqrt(cc * cc + 4.0 * sq);
      const double sg = j == np ? 1.0 : -1.0;
      x = sg * cc >= 0.0 ? 0.5 * (cc + sg * rt) - tau : -2.0 * sq / (cc - sg * rt) - tau;
    } else {
      // c + e / (0 - x) = 0 fitted at tau: e = g' tau^2, c = g + g' tau
      x = dg * tau * tau / (g + dg * tau) - tau;
    }
    double tn = mid;
    if (x == x) {
      // a model step at the rounding level of tau: converged (tau has just
      // become an end of the bracket, so it must not be tested against it)
      if (fabs(x) <= 2.0 * kU * fabs(tau)) {
        lo = hi = tau;
        break;
      }
      tn = tau + x;
    }
    if (!(tn > lo && tn < hi)) tn = mid;
    const double step = fabs(tn - tau);
    tau = tn;
    if (step <= 2.0 * kU * fabs(tn)) {
      lo = hi = tn;
      break;
    }
  }
  if (lane == 0) {
    s.ro[j] = o;
    s.rt[j] = lo == hi ? lo : 0.5 * (lo + hi);
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
// One wavefront per pole: the lanes share the product over k.
template <bool ARROW>
__global__ __launch_bounds__(256) void k_lowner(Sec s0, int S, const double* __restrict__ a_or_rho) {
  const int b = blockIdx.y;
  const Sec s = sec_at(s0, b, S);
  const int np = s.cnt[0];
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= np) return;
  const double* p = s.p;
  const double pi = p[i];
  // ARROW: f_i^2 = -(p_i - l_i)(p_i - l_{i+1}) prod_{k<i} (p_i - l_k)/(p_i - p_k)
  //                                            prod_{k>i} (p_i - l_{k+1})/(p_i - p_k)
  // RANK1: z_i^2 = -(1/rho)(d_i - l_{n-1}) prod_{k<i} (d_i - l_k)/(d_i - d_k)
  //                                       prod_{k>i} (d_i - l_{k-1})/(d_i - d_k)
  double prod = 1.0;
  for (int k = lane; k < np; k += 64) {
    if (k < i) prod *= (-lam_minus(s, k, i)) / (pi - p[k]);
    else if (k > i) prod *= (-lam_minus(s, ARROW ? k + 1 : k - 1, i)) / (pi - p[k]);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) prod *= __shfl_xor(prod, off, 64);
  if (lane == 0) {
    const double lead = ARROW ? -(lam_minus(s, i, i) * lam_minus(s, i + 1, i))  // (l_i - p_i)(l_{i+1} - p_i) < 0
                              : lam_minus(s, np - 1, i) / a_or_rho[b];          // (l_{n-1} - d_i)/rho > 0
    const double sign = s.what[i] < 0.0 ? -1.0 : 1.0;
    s.what[i] = sign * sqrt(fmax(lead * prod, 0.0));
  }
}

// Ascending order of the eigenvalues: the secular roots (ascending by
// construction) and the deflated values (ascending: k_deflate writes them in
// index order).  Every value finds its position by binary search in the other
// list (roots first on ties).  Writes lam[position] and pos[source] =
// position, source = root r or nroots + q for the q-th deflated value.
template <bool ARROW>
__global__ __launch_bounds__(256) void k_order(Sec s0, int S, double* __restrict__ lam, int64_t lstride,
                                               int* __restrict__ pos, int64_t pstride) {
  const int b = blockIdx.x;
  const Sec s = sec_at(s0, b, S);
  const int np = s.cnt[0], nd = s.cnt[2];
  const int nroots = ARROW ? np + 1 : np;
  const double* dv = s.dval;
  double* lb = lam + (int64_t)b * lstride;
  int* pb = pos + (int64_t)b * pstride;
  for (int r = threadIdx.x; r < nroots; r += blockDim.x) {
    const double v = root_val(s, r);
    int lo = 0, hi = nd;  // number of deflated values < v
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (dv[mid] < v) lo = mid + 1; else hi = mid;
    }
    lb[r + lo] = v;
    pb[r] = r + lo;
  }
  for (int q = threadIdx.x; q < nd; q += blockDim.x) {
    const double v = dv[q];
    int lo = 0, hi = nroots;  // number of roots <= v
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (root_val(s, mid) <= v) lo = mid + 1; else hi = mid;
    }
    lb[q + lo] = v;
    pb[nroots + q] = q + lo;
  }
}

// Eigenvector of root j (one block per root, grid.y = problem), written as
// column pos[j] of X (ldx rows, row index space of the problem).  ARROW:
// entries at the pole rows and 1 at the tip row; RANK1: entries at the pole
// rows.  X must be zero beforehand.
template <bool ARROW>
__global__ __launch_bounds__(256) void k_vectors(Sec s0, int S, const int* __restrict__ pos, int64_t pstride,
                                                 double* __restrict__ x, int64_t xstride, int ldx, int tip_row) {
  const int b = blockIdx.y;
  const Sec s = sec_at(s0, b, S);
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
  double* col = x + (int64_t)b * xstride + (int64_t)pos[(int64_t)b * pstride + j] * ldx;
  for (int i = threadIdx.x; i < np; i += blockDim.x) {
    const double den = ARROW ? lam_minus(s, j, i) : -lam_minus(s, j, i);
    col[s.idx[i]] = s.what[i] / den / nrm;
  }
  if (ARROW && threadIdx.x == 0) col[tip_row] = 1.0 / nrm;
}

// deflated columns: unit vectors at their rows, in their ordered columns
template <bool ARROW>
__global__ void k_deflated_cols(Sec s0, int S, const int* __restrict__ pos, int64_t pstride,
                                double* __restrict__ x, int64_t xstride, int ldx) {
  const int b = blockIdx.y;
  const Sec s = sec_at(s0, b, S);
  const int nd = s.cnt[2];
  const int nroots = ARROW ? s.cnt[0] + 1 : s.cnt[0];
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nd) return;
  x[(int64_t)b * xstride + (int64_t)pos[(int64_t)b * pstride + nroots + q] * ldx + s.didx[q]] = 1.0;
}

// undo the deflation rotations on the rows of X (latest first), all columns
__global__ void k_unrotate(Sec s0, int S, double* __restrict__ x, int64_t xstride, int ldx, int ncols) {
  const int b = blockIdx.x;
  const Sec s = sec_at(s0, b, S);
  const int nr = s.cnt[1];
  double* xb = x + (int64_t)b * xstride;
  for (int r = nr - 1; r >= 0; --r) {
    const int pi = s.rot_i[r], pj = s.rot_j[r];
    const double c = s.rot_c[r], sn = s.rot_s[r];
    for (int col = threadIdx.x; col < ncols; col += blockDim.x) {
      double* xc = xb + (int64_t)col * ldx;
      const double a = xc[pi], bb = xc[pj];
      xc[pi] = c * a + sn * bb;
      xc[pj] = -sn * a + c * bb;
    }
    __syncthreads();
  }
}

// -------------------------------------------------------------------------
// tears, leaves, merges
// -------------------------------------------------------------------------

// SVD of a D x D matrix g (column-major) by one-sided Jacobi: g = P S Q^T.
// Columns of P with s = 0 are returned as zero (their rank-one update has
// rho = 0 and deflates whatever its coupling).  D is a template parameter so
// that the unrolled loops keep the matrices in registers.
template <int D>
__device__ void svd_small(const double* g, double* pm, double* sv, double* qm) {
  double a[D * D], v[D * D];
#pragma unroll
  for (int i = 0; i < D * D; ++i) {
    a[i] = g[i];
    v[i] = (i % D) == (i / D) ? 1.0 : 0.0;
  }
  for (int sweep = 0; sweep < 40; ++sweep) {
    bool rotated = false;
#pragma unroll
    for (int k = 0; k < D - 1; ++k)
#pragma unroll
      for (int l = k + 1; l < D; ++l) {
        double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
        for (int r = 0; r < D; ++r) {
          al += a[r + k * D] * a[r + k * D];
          be += a[r + l * D] * a[r + l * D];
          ga += a[r + k * D] * a[r + l * D];
        }
        if (ga != 0.0 && fabs(ga) > 4.0 * kU * sqrt(al * be)) {
          rotated = true;
          const double ze = (be - al) / (2.0 * ga);
          const double t = (ze >= 0.0 ? 1.0 : -1.0) / (fabs(ze) + sqrt(1.0 + ze * ze));
          const double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
#pragma unroll
          for (int r = 0; r < D; ++r) {
            const double x = a[r + k * D], y = a[r + l * D];
            a[r + k * D] = c * x - sn * y;
            a[r + l * D] = sn * x + c * y;
            const double vx = v[r + k * D], vy = v[r + l * D];
            v[r + k * D] = c * vx - sn * vy;
            v[r + l * D] = sn * vx + c * vy;
          }
        }
      }
    if (!rotated) break;
  }
#pragma unroll
  for (int k = 0; k < D; ++k) {
    double nr = 0.0;
#pragma unroll
    for (int r = 0; r < D; ++r) nr += a[r + k * D] * a[r + k * D];
    nr = sqrt(nr);
    sv[k] = nr;
#pragma unroll
    for (int r = 0; r < D; ++r) {
      pm[r + k * D] = nr > 0.0 ? a[r + k * D] / nr : 0.0;
      qm[r + k * D] = v[r + k * D];
    }
  }
}

// Eigen-decomposition of a symmetric D x D matrix (cyclic Jacobi), eigenvalues
// ascending with their vectors (u column-major).
template <int D>
__device__ void eig_small(double (&a)[D * D], double* lam, double* u) {
  double v[D * D];
#pragma unroll
  for (int i = 0; i < D * D; ++i) v[i] = (i % D) == (i / D) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 50; ++sweep) {
    double off = 0.0, tot = 0.0;
#pragma unroll
    for (int i = 0; i < D * D; ++i) {
      tot += a[i] * a[i];
      if ((i % D) != (i / D)) off += a[i] * a[i];
    }
    if (off == 0.0 || off <= 16.0 * kU * kU * tot) break;
#pragma unroll
    for (int k = 0; k < D - 1; ++k)
#pragma unroll
      for (int l = k + 1; l < D; ++l) {
        const double akl = a[k + l * D];
        if (akl != 0.0) {
          const double th = (a[l + l * D] - a[k + k * D]) / (2.0 * akl);
          const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
          const double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
          // A <- J^T A J with J the rotation in the plane (k, l)
#pragma unroll
          for (int r = 0; r < D; ++r) {
            const double x = a[r + k * D], y = a[r + l * D];
            a[r + k * D] = c * x - sn * y;
            a[r + l * D] = sn * x + c * y;
          }
#pragma unroll
          for (int r = 0; r < D; ++r) {
            const double x = a[k + r * D], y = a[l + r * D];
            a[k + r * D] = c * x - sn * y;
            a[l + r * D] = sn * x + c * y;
          }
#pragma unroll
          for (int r = 0; r < D; ++r) {
            const double x = v[r + k * D], y = v[r + l * D];
            v[r + k * D] = c * x - sn * y;
            v[r + l * D] = sn * x + c * y;
          }
        }
      }
  }
  // selection order of the diagonal (D is small), ties by index
#pragma unroll
  for (int i = 0; i < D; ++i) {
    int rank = 0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const double aj = a[j + j * D], ai = a[i + i * D];
      rank += (aj < ai || (aj == ai && j < i)) ? 1 : 0;
    }
    lam[rank] = a[i + i * D];
#pragma unroll
    for (int r = 0; r < D; ++r) u[r + rank * D] = v[r + i * D];
  }
}

// Tears of the couplings.  Slot t holds P (d x d), S (d), Q (d x d) of the
// coupling between chain blocks t and t+1; chain block 0 is the first block
// listed in gam (gam + t d^2 is the coupling of chain blocks t, t+1).
// Slots t >= nreal are decoupled padding: S = 0, P = 0, Q = I.
template <int D>
__global__ __launch_bounds__(64) void k_tear(int nslots, int nreal, const double* __restrict__ gam, double* __restrict__ pm,
                       double* __restrict__ sv, double* __restrict__ qm) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nslots) return;
  double* p = pm + (int64_t)t * D * D;
  double* q = qm + (int64_t)t * D * D;
  double* s = sv + (int64_t)t * D;
  if (t < nreal) {
    svd_small<D>(gam + (int64_t)t * D * D, p, s, q);
  } else {
#pragma unroll
    for (int c = 0; c < D; ++c) {
      s[c] = 0.0;
#pragma unroll
      for (int r = 0; r < D; ++r) {
        p[r + c * D] = 0.0;
        q[r + c * D] = r == c ? 1.0 : 0.0;
      }
    }
  }
}

// Leaves of the tail: block t (0-based within the tail, first tail block at
// xi0) minus Q S Q^T of the tear below it (slot toff + t) and P S P^T of the
// tear above it (slot toff + t - 1, which for t = 0 exists only when toff =
// 1: the tear between the arrowhead and the tail).  Blocks t >= nb are
// decoupled padding with eigenvalues big + t d + i.
template <int D>
__global__ __launch_bounds__(64) void k_leaf(int nb, int nb2, int toff, double big, const double* __restrict__ xi0,
                       const double* __restrict__ pm, const double* __restrict__ sv,
                       const double* __restrict__ qm, double* __restrict__ lam, double* __restrict__ u) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nb2) return;
  double* lt = lam + (int64_t)t * D;
  double* ut = u + (int64_t)t * D * D;
  if (t >= nb) {
#pragma unroll
    for (int c = 0; c < D; ++c) {
      lt[c] = big + (double)(t * D + c);
#pragma unroll
      for (int r = 0; r < D; ++r) ut[r + c * D] = r == c ? 1.0 : 0.0;
    }
    return;
  }
  double a[D * D];
#pragma unroll
  for (int i = 0; i < D * D; ++i) a[i] = xi0[(int64_t)t * D * D + i];
  const int below = toff + t, above = toff + t - 1;
  if (t < nb - 1) {
    const double* q = qm + (int64_t)below * D * D;
    const double* s = sv + (int64_t)below * D;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const double sk = s[k];
#pragma unroll
      for (int c = 0; c < D; ++c)
#pragma unroll
        for (int r = 0; r < D; ++r) a[r + c * D] -= q[r + k * D] * sk * q[c + k * D];
    }
  }
  if (above >= 0) {
    const double* p = pm + (int64_t)above * D * D;
    const double* s = sv + (int64_t)above * D;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const double sk = s[k];
#pragma unroll
      for (int c = 0; c < D; ++c)
#pragma unroll
        for (int r = 0; r < D; ++r) a[r + c * D] -= p[r + k * D] * sk * p[c + k * D];
    }
  }
  // The corrections round differently in (r, c) and (c, r).  Jacobi's stopping
  // test (off-diagonal mass below 16 u^2 of the total) cannot be met while the
  // block is asymmetric at that level, and such leaves ran all 50 sweeps.
#pragma unroll
  for (int c = 1; c < D; ++c)
#pragma unroll
    for (int r = 0; r < c; ++r) {
      const double m = 0.5 * (a[r + c * D] + a[c + r * D]);
      a[r + c * D] = m;
      a[c + r * D] = m;
    }
  eig_small<D>(a, lt, ut);
}

// arrow tip block X = Xi_{l0+1} - Q S Q^T of the tear with the tail (slot 0)
__global__ void k_tip(int d, const double* __restrict__ xi1, const double* __restrict__ qm,
                      const double* __restrict__ sv, int has_tail, double* __restrict__ x) {
  const int e = threadIdx.x;
  if (e >= d * d) return;
  const int r = e % d, c = e / d;
  double acc = 0.0;
  if (has_tail)
    for (int k = 0; k < d; ++k) acc += qm[r + k * d] * sv[k] * qm[c + k * d];
  x[e] = xi1[e] - acc;
}

// Union of two ascending lists (left first on ties), one block per problem:
// poles[position] = value, src[position] = a (left) or mL + r (right).
__global__ void k_union(int mL, int mR, const double* __restrict__ lamL, int64_t sL,
                        const double* __restrict__ lamR, int64_t sR, double* __restrict__ poles,
                        int* __restrict__ src, int64_t so) {
  const int b = blockIdx.x;
  const double* l = lamL + (int64_t)b * sL;
  const double* r = lamR + (int64_t)b * sR;
  double* po = poles + (int64_t)b * so;
  int* sr = src + (int64_t)b * so;
  for (int a = threadIdx.x; a < mL; a += blockDim.x) {
    const double v = l[a];
    int lo = 0, hi = mR;  // right values < v
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (r[mid] < v) lo = mid + 1; else hi = mid;
    }
    po[a + lo] = v;
    sr[a + lo] = a;
  }
  for (int c = threadIdx.x; c < mR; c += blockDim.x) {
    const double v = r[c];
    int lo = 0, hi = mL;  // left values <= v
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (l[mid] <= v) lo = mid + 1; else hi = mid;
    }
    po[c + lo] = v;
    sr[c + lo] = mL + c;
  }
}

// Coupling vector of the first update of a merge, in the union order: z[k] =
// U_L(last d rows, col) q (left columns) or U_R(first d rows, col) p (right
// columns), with q = Q(:, i), p = P(:, i) of the problem's tear slot
// (slot0 + b sstep); also rho[b] = S(i).
__global__ void k_zfirst(int mL, int mR, int d, int i, const double* __restrict__ uL, int64_t suL, int ldL,
                         const double* __restrict__ uR, int64_t suR, int ldR, const int* __restrict__ src,
                         int64_t so, const double* __restrict__ pm, const double* __restrict__ sv,
                         const double* __restrict__ qm, int slot0, int sstep, double* __restrict__ z,
                         double* __restrict__ rho) {
  const int b = blockIdx.y;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int slot = slot0 + b * sstep;
  if (k == 0) rho[b] = sv[(int64_t)slot * d + i];
  if (k >= mL + mR) return;
  const int sc = src[(int64_t)b * so + k];
  double acc = 0.0;
  if (sc < mL) {
    const double* col = uL + (int64_t)b * suL + (int64_t)sc * ldL + (mL - d);
    const double* q = qm + (int64_t)slot * d * d + (int64_t)i * d;
    for (int r = 0; r < d; ++r) acc += col[r] * q[r];
  } else {
    const double* col = uR + (int64_t)b * suR + (int64_t)(sc - mL) * ldR;
    const double* p = pm + (int64_t)slot * d * d + (int64_t)i * d;
    for (int r = 0; r < d; ++r) acc += col[r] * p[r];
  }
  z[(int64_t)b * (mL + mR) + k] = acc;
}

// Coupling vector of a later update of a merge: z = E^T v, v = q_i at rows
// mL-d..mL-1 and p_i at rows mL..mL+d-1 of E (m x m, ld ldE); rho[b] = S(i).
__global__ void k_zvec(int m, int mL, int d, int i, const double* __restrict__ e, int64_t se, int ldE,
                       const double* __restrict__ pm, const double* __restrict__ sv,
                       const double* __restrict__ qm, int slot0, int sstep, double* __restrict__ z,
                       double* __restrict__ rho) {
  const int b = blockIdx.y;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int slot = slot0 + b * sstep;
  if (k == 0) rho[b] = sv[(int64_t)slot * d + i];
  if (k >= m) return;
  const double* col = e + (int64_t)b * se + (int64_t)k * ldE;
  const double* q = qm + (int64_t)slot * d * d + (int64_t)i * d;
  const double* p = pm + (int64_t)slot * d * d + (int64_t)i * d;
  double acc = 0.0;
  for (int r = 0; r < d; ++r) acc += col[mL - d + r] * q[r] + col[mL + r] * p[r];
  z[(int64_t)b * m + k] = acc;
}

// split the rows of the merge eigenvectors W (m x m, rows in union order) by
// the block they came from: Wl (mL x m, row = left column) and Wr (mR x m)
__global__ void k_split(int m, int mL, const double* __restrict__ w, int64_t sw, const int* __restrict__ src,
                        int64_t so, double* __restrict__ wl, int64_t sl, double* __restrict__ wr,
                        int64_t sr) {
  const int b = blockIdx.y;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)m * m) return;
  const int k = (int)(e % m), j = (int)(e / m);
  const double v = w[(int64_t)b * sw + e];
  const int sc = src[(int64_t)b * so + k];
  const int mR = m - mL;
  if (sc < mL) wl[(int64_t)b * sl + (int64_t)j * mL + sc] = v;
  else wr[(int64_t)b * sr + (int64_t)j * mR + (sc - mL)] = v;
}

// border row i of the block arrowhead in the current row space (kk + i rows):
// c = [F(i, :), X(i, 0:i)]
__global__ void k_arrow_c(int kk, int d, int i, const double* __restrict__ f, const double* __restrict__ x,
                          double* __restrict__ c) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= kk + i) return;
  c[k] = k < kk ? f[i + (int64_t)k * d] : x[i + (int64_t)(k - kk) * d];
}

// row m of E (ld m + 1) = row m of W (ld m + 1): the new tip row
__global__ void k_copy_row(int m, const double* __restrict__ w, double* __restrict__ e) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j > m) return;
  e[m + (int64_t)j * (m + 1)] = w[m + (int64_t)j * (m + 1)];
}

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct EigWork {
  DBuf b_int, b_dbl, b_tear, b_small, b_lam, b_g0, b_g1, b_g2, b_w, b_wl, b_wr, b_ea, b_eb, b_c;
};

namespace {

Sec make_sec(double*& dp, int*& ip, int nbat, int S) {
  Sec s;
  const int64_t n = (int64_t)nbat * S;
  s.cnt = ip; ip += 4 * nbat;
  s.p = dp; dp += n;
  s.w = dp; dp += n;
  s.idx = ip; ip += n;
  s.rot_i = ip; ip += n;
  s.rot_j = ip; ip += n;
  s.rot_c = dp; dp += n;
  s.rot_s = dp; dp += n;
  s.dval = dp; dp += n;
  s.didx = ip; ip += n;
  s.ro = ip; ip += n;
  s.rt = dp; dp += n;
  s.what = dp; dp += n;
  return s;
}
constexpr int kSecDbl = 7, kSecInt = 6;  // per-entry doubles / ints of a Sec (plus 4 ints per problem)

void gemm_batched(nsp_ctx* c, int m, int n, int k, const double* a, int lda, int64_t sa, const double* b,
                  int ldb, int64_t sb, double* cc, int ldc, int64_t sc, int batch) {
  const double one = 1.0, zero = 0.0;
  if (batch == 1) {
    NSP_BLAS(rocblas_dgemm(c->blas, rocblas_operation_none, rocblas_operation_none, m, n, k, &one, a, lda,
                           b, ldb, &zero, cc, ldc));
  } else {
    NSP_BLAS(rocblas_dgemm_strided_batched(c->blas, rocblas_operation_none, rocblas_operation_none, m, n, k,
                                           &one, a, lda, sa, b, ldb, sb, &zero, cc, ldc, sc, batch));
  }
}

// One secular solve per problem of a batch, eigenvectors into X (zeroed here,
// columns ascending), eigenvalues into lam.  RANK1 problems: m poles (vals
// ascending), couplings cpl, rho per problem; ARROW: m poles, tip per problem,
// X has m + 1 rows and columns.
template <bool ARROW>
void secular(nsp_ctx* c, Sec sec, int S, int nbat, int m, const double* vals, int64_t vstride,
             const double* cpl, int cinc, int64_t cstride, const double* a_or_rho, double scale,
             double bound, double* lam, int64_t lstride, int* pos, int64_t pstride, double* x,
             int64_t xstride, int ldx) {
  const int nroots = ARROW ? m + 1 : m;
  const size_t lds2 = sizeof(double) * 2 * (size_t)m;
  const bool lds = lds2 <= (size_t)kLdsBytes;
  const size_t lds_d = (2 * sizeof(int) + 1) * (size_t)m + 16;
  if (lds_d > (size_t)kLdsBytes) throw Error(NSP_ERR_ARG, "restart matrix too large for the eigensolver");
  k_deflate<<<nbat, kDeflThreads, lds_d, c->stream>>>(m, vals, vstride, cpl, cinc, cstride,
                                                      ARROW ? nullptr : a_or_rho, scale, sec, S);
  const dim3 gr(nb(nroots, 4), nbat);
  if (lds)
    k_roots<ARROW, true><<<gr, 256, lds2, c->stream>>>(sec, S, a_or_rho, -bound, bound);
  else
    k_roots<ARROW, false><<<gr, 256, 0, c->stream>>>(sec, S, a_or_rho, -bound, bound);
  k_lowner<ARROW><<<dim3(nb(m, 4), nbat), 256, 0, c->stream>>>(sec, S, a_or_rho);
  k_order<ARROW><<<nbat, 256, 0, c->stream>>>(sec, S, lam, lstride, pos, pstride);
  const int xc = ARROW ? m + 1 : m;
  if (nbat == 1 || xstride == (int64_t)ldx * xc) {
    NSP_HIP(hipMemsetAsync(x, 0, sizeof(double) * (size_t)ldx * xc * nbat, c->stream));
  } else {
    NSP_HIP(hipMemset2DAsync(x, sizeof(double) * (size_t)xstride, 0, sizeof(double) * (size_t)ldx * xc, nbat,
                             c->stream));
  }
  k_vectors<ARROW><<<dim3(nroots, nbat), 256, 0, c->stream>>>(sec, S, pos, pstride, x, xstride, ldx, m);
  k_deflated_cols<ARROW><<<dim3(nb(m + 1, 256), nbat), 256, 0, c->stream>>>(sec, S, pos, pstride, x,
                                                                             xstride, ldx);
  k_unrotate<<<nbat, 1024, 0, c->stream>>>(sec, S, x, xstride, ldx, xc);
  NSP_HIP(hipGetLastError());
}

inline int next_pow2(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

}  // namespace

// Eigen-decomposition of T (see the file comment).  xi and gam are indexed by
// Lanczos block number (block j at xi + j d^2, column-major d x d; gam + j d^2
// is the coupling of blocks j and j+1, i.e. T(block j+1, block j)); theta and
// f (d x kk, column-major) hold the kk kept Ritz values and their coupling.
// norm_t bounds ||T||.  On return evecs (K x K, column-major) holds the
// eigenvectors and evals the eigenvalues, ascending.
void eig_restart(nsp_ctx* c, EigWork& w, int K, int d, int kk, double norm_t, const double* theta,
                 const double* f, const double* xi, const double* gam, double* evals, double* evecs) {
  const int L = K / d, l0 = kk / d;
  if (K % d || kk % d || kk > K - d || L < 1) throw Error(NSP_ERR_ARG, "eig_restart: inconsistent sizes");
  const bool arrow = kk > 0;
  const int jb0 = arrow ? l0 + 2 : 1;      // first tail block (Lanczos block number)
  const int nbt = L - jb0 + 1;             // tail blocks (0 when the arrowhead is all of T)
  const int m1 = arrow ? kk + d : 0, m2 = nbt * d;
  const int nb2 = nbt > 0 ? next_pow2(nbt) : 0, m2p = nb2 * d;
  const int toff = arrow ? 1 : 0;          // tear slot 0: arrowhead-tail (when both exist)
  const int nslots = toff + std::max(nb2 - 1, 0);
  const double big = 4.0 * norm_t + 4.0;   // above every eigenvalue of every sub-problem
  const double bound = 4.0 * norm_t + 1.0; // every arrowhead eigenvalue lies inside
  const int mmax = std::max(K, m2p) + 2;

  // workspaces (sized by K so that they are allocated once per run)
  const int64_t big2 = (int64_t)mmax * mmax;
  w.b_dbl.alloc(sizeof(double) * (size_t)(kSecDbl * (2 * mmax + 64) + 6 * mmax + 64));
  w.b_int.alloc(sizeof(int) * (size_t)(kSecInt * (2 * mmax + 64) + 4 * (mmax + 64) + 3 * mmax + 64));
  w.b_tear.alloc(sizeof(double) * (size_t)(std::max(nslots, 1) * (2 * d * d + d)));
  w.b_small.alloc(sizeof(double) * (size_t)(kMaxD * kMaxD + 2 * mmax + 64));
  w.b_lam.alloc(sizeof(double) * (size_t)(3 * mmax));
  w.b_g0.alloc(sizeof(double) * (size_t)big2);
  w.b_g1.alloc(sizeof(double) * (size_t)big2);
  w.b_g2.alloc(sizeof(double) * (size_t)big2);
  w.b_w.alloc(sizeof(double) * (size_t)big2);
  w.b_wl.alloc(sizeof(double) * (size_t)big2);
  w.b_wr.alloc(sizeof(double) * (size_t)big2);
  double* pm = w.b_tear.as<double>();
  double* qm = pm + (int64_t)std::max(nslots, 1) * d * d;
  double* sv = qm + (int64_t)std::max(nslots, 1) * d * d;
  double* xtip = w.b_small.as<double>();
  double* rho = xtip + kMaxD * kMaxD;
  double* zc = rho + mmax + 32;  // coupling vectors (z), up to mmax
  double* lamb[3] = {w.b_lam.as<double>(), w.b_lam.as<double>() + mmax, w.b_lam.as<double>() + 2 * mmax};
  double* dp0 = w.b_dbl.as<double>();
  int* ip0 = w.b_int.as<int>();
  double* poles = dp0 + kSecDbl * (2 * mmax + 64);
  double* zb = poles + mmax;        // batched coupling vectors
  int* src = ip0 + kSecInt * (2 * mmax + 64);
  int* pos = src + mmax;

  // ---- tears and leaves
  if (nslots > 0) {
    // slot 0 (arrow case): Gamma_{l0+1}; tail slots: Gamma_{jb0 + t}
    const int nreal = arrow ? nbt : std::max(nbt - 1, 0);  // couplings present in gam
    const double* g0 = gam + (int64_t)(arrow ? l0 + 1 : 1) * d * d;
    switch (d) {
      case 1: k_tear<1><<<nb(nslots, 64), 64, 0, c->stream>>>(nslots, nreal, g0, pm, sv, qm); break;
      case 2: k_tear<2><<<nb(nslots, 64), 64, 0, c->stream>>>(nslots, nreal, g0, pm, sv, qm); break;
      case 4: k_tear<4><<<nb(nslots, 64), 64, 0, c->stream>>>(nslots, nreal, g0, pm, sv, qm); break;
      case 8: k_tear<8><<<nb(nslots, 64), 64, 0, c->stream>>>(nslots, nreal, g0, pm, sv, qm); break;
      default: throw Error(NSP_ERR_ARG, "eig_restart: d must be 1, 2, 4 or 8");
    }
    NSP_HIP(hipGetLastError());
  }

  // ---- tail: leaves, then merges level by level (E groups in b_g0/b_g1)
  double* tl_lam = nullptr;  // tail eigenvalues (m2p, ascending, the first m2 real)
  double* tl_vec = nullptr;  // tail eigenvectors (m2p x m2p, ld m2p)
  if (nbt > 0) {
    double* gcur = w.b_g0.as<double>();
    double* gnext = w.b_g1.as<double>();
    double* gtmp = w.b_g2.as<double>();
    double* lcur = lamb[0];
    double* lnext = lamb[1];
    double* ltmp = lamb[2];
    const double* xi0 = xi + (int64_t)jb0 * d * d;
    switch (d) {
      case 1: k_leaf<1><<<nb(nb2, 64), 64, 0, c->stream>>>(nbt, nb2, toff, big, xi0, pm, sv, qm, lcur, gcur); break;
      case 2: k_leaf<2><<<nb(nb2, 64), 64, 0, c->stream>>>(nbt, nb2, toff, big, xi0, pm, sv, qm, lcur, gcur); break;
      case 4: k_leaf<4><<<nb(nb2, 64), 64, 0, c->stream>>>(nbt, nb2, toff, big, xi0, pm, sv, qm, lcur, gcur); break;
      case 8: k_leaf<8><<<nb(nb2, 64), 64, 0, c->stream>>>(nbt, nb2, toff, big, xi0, pm, sv, qm, lcur, gcur); break;
      default: throw Error(NSP_ERR_ARG, "eig_restart: d must be 1, 2, 4 or 8");
    }
    NSP_HIP(hipGetLastError());
    for (int gs = d, lev = 0; gs < m2p; gs *= 2, ++lev) {
      const int m = 2 * gs, npair = m2p / m;
      const int S = m + 2;
      double* dp = dp0;
      int* ip = ip0;
      Sec sec = make_sec(dp, ip, npair, S);
      // tear slot of pair b: the coupling between tail blocks (2b+1) 2^lev - 1 and (2b+1) 2^lev
      const int slot0 = toff + (1 << lev) - 1, sstep = 1 << (lev + 1);
      const int64_t sg = (int64_t)gs * gs, sm = (int64_t)m * m;
      // first update: union of the children's spectra, block-structured GEMMs
      k_union<<<npair, 256, 0, c->stream>>>(gs, gs, lcur, m, lcur + gs, m, poles, src, m);
      k_zfirst<<<dim3(nb(m, 256), npair), 256, 0, c->stream>>>(gs, gs, d, 0, gcur, 2 * sg, gs, gcur + sg,
                                                              2 * sg, gs, src, m, pm, sv, qm, slot0, sstep,
                                                              zb, rho);
      NSP_HIP(hipGetLastError());
      double* wbuf = w.b_w.as<double>();
      secular<false>(c, sec, S, npair, m, poles, m, zb, 1, m, rho, norm_t, bound, lnext, m, pos, m, wbuf, sm, m);
      double* wl = w.b_wl.as<double>();
      double* wr = w.b_wr.as<double>();
      k_split<<<dim3(nb(sm, 256), npair), 256, 0, c->stream>>>(m, gs, wbuf, sm, src, m, wl, (int64_t)gs * m,
                                                              wr, (int64_t)gs * m);
      NSP_HIP(hipGetLastError());
      gemm_batched(c, gs, m, gs, gcur, gs, 2 * sg, wl, gs, (int64_t)gs * m, gnext, m, sm, npair);
      gemm_batched(c, gs, m, gs, gcur + sg, gs, 2 * sg, wr, gs, (int64_t)gs * m, gnext + gs, m, sm, npair);
      // later updates: dense
      for (int i = 1; i < d; ++i) {
        k_zvec<<<dim3(nb(m, 256), npair), 256, 0, c->stream>>>(m, gs, d, i, gnext, sm, m, pm, sv, qm, slot0,
                                                              sstep, zb, rho);
        NSP_HIP(hipGetLastError());
        secular<false>(c, sec, S, npair, m, lnext, m, zb, 1, m, rho, norm_t, bound, ltmp, m, pos, m, wbuf, sm,
                       m);
        gemm_batched(c, m, m, m, gnext, m, sm, wbuf, m, sm, gtmp, m, sm, npair);
        std::swap(gnext, gtmp);
        std::swap(lnext, ltmp);
      }
      std::swap(gcur, gnext);
      std::swap(lcur, lnext);
    }
    tl_lam = lcur;
    tl_vec = gcur;
    // keep the tail's buffers out of the way of what follows
    if (tl_vec != w.b_g0.as<double>()) {
      NSP_HIP(hipMemcpyAsync(w.b_g0.as<double>(), tl_vec, sizeof(double) * (size_t)m2p * m2p,
                             hipMemcpyDeviceToDevice, c->stream));
      tl_vec = w.b_g0.as<double>();
    }
    if (tl_lam != lamb[0]) {
      NSP_HIP(hipMemcpyAsync(lamb[0], tl_lam, sizeof(double) * (size_t)m2p, hipMemcpyDeviceToDevice,
                             c->stream));
      tl_lam = lamb[0];
    }
  }

  if (!arrow) {
    // first cycle: T is the tail (m2 = K); copy the real block out
    NSP_HIP(hipMemcpy2DAsync(evecs, sizeof(double) * K, tl_vec, sizeof(double) * m2p, sizeof(double) * K, K,
                             hipMemcpyDeviceToDevice, c->stream));
    NSP_HIP(hipMemcpyAsync(evals, tl_lam, sizeof(double) * K, hipMemcpyDeviceToDevice, c->stream));
    return;
  }

  // ---- block arrowhead M1 = [diag(theta) F^T; F X], X = Xi_{l0+1} - Q S Q^T
  k_tip<<<1, 64, 0, c->stream>>>(d, xi + (int64_t)(l0 + 1) * d * d, qm, sv, nbt > 0 ? 1 : 0, xtip);
  NSP_HIP(hipGetLastError());
  double* ea = w.b_g1.as<double>();   // current arrowhead eigenvectors ((kk+i) x (kk+i), compact)
  double* eb = w.b_g2.as<double>();
  double* la = lamb[1];
  double* lb2 = lamb[2];
  {
    const int m = kk, S = m + 3;
    double* dp = dp0;
    int* ip = ip0;
    Sec sec = make_sec(dp, ip, 1, S);
    // first tip: poles theta, couplings F(0, :), tip X(0, 0); eigenvectors = W
    secular<true>(c, sec, S, 1, m, theta, 0, f, d, 0, xtip, norm_t, bound, la, 0, pos, 0, ea, 0, m + 1);
    for (int i = 1; i < d; ++i) {
      const int mi = kk + i, Si = mi + 3;
      dp = dp0;
      ip = ip0;
      Sec si = make_sec(dp, ip, 1, Si);
      k_arrow_c<<<nb(mi, 256), 256, 0, c->stream>>>(kk, d, i, f, xtip, zc);
      NSP_HIP(hipGetLastError());
      const double one = 1.0, zero = 0.0;
      // z = E^T c
      NSP_BLAS(rocblas_dgemv(c->blas, rocblas_operation_transpose, mi, mi, &one, ea, mi, zc, 1, &zero, zb, 1));
      double* wbuf = w.b_w.as<double>();
      secular<true>(c, si, Si, 1, mi, la, 0, zb, 1, 0, xtip + i + (int64_t)i * d, norm_t, bound, lb2, 0, pos,
                    0, wbuf, 0, mi + 1);
      // E_new = [E 0; 0 1] W: rows 0..mi-1 by GEMM, row mi copied
      NSP_BLAS(rocblas_dgemm(c->blas, rocblas_operation_none, rocblas_operation_none, mi, mi + 1, mi, &one, ea,
                             mi, wbuf, mi + 1, &zero, eb, mi + 1));
      k_copy_row<<<nb(mi + 1, 256), 256, 0, c->stream>>>(mi, wbuf, eb);
      NSP_HIP(hipGetLastError());
      std::swap(ea, eb);
      std::swap(la, lb2);
    }
  }

  // ---- join arrowhead (m1) and tail (m2) with the d updates of tear slot 0
  {
    const int m = K, S = m + 2;
    double* dp = dp0;
    int* ip = ip0;
    Sec sec = make_sec(dp, ip, 1, S);
    double* lf = lb2;  // free eigenvalue buffer (la holds the arrowhead's)
    k_union<<<1, 256, 0, c->stream>>>(m1, m2, la, 0, tl_lam, 0, poles, src, 0);
    k_zfirst<<<dim3(nb(m, 256), 1), 256, 0, c->stream>>>(m1, m2, d, 0, ea, 0, m1, tl_vec, 0, m2p, src, 0, pm,
                                                         sv, qm, 0, 0, zb, rho);
    NSP_HIP(hipGetLastError());
    double* wbuf = w.b_w.as<double>();
    secular<false>(c, sec, S, 1, m, poles, 0, zb, 1, 0, rho, norm_t, bound, lf, 0, pos, 0, wbuf, 0, m);
    double* wl = w.b_wl.as<double>();
    double* wr = w.b_wr.as<double>();
    k_split<<<dim3(nb((int64_t)m * m, 256), 1), 256, 0, c->stream>>>(m, m1, wbuf, 0, src, 0, wl, 0, wr, 0);
    NSP_HIP(hipGetLastError());
    // the final eigenvectors go to evecs after an odd number of dense updates
    // behind the first, to eb otherwise, so that the last lands in evecs
    double* cur = (d % 2 == 1) ? evecs : eb;
    double* other = (d % 2 == 1) ? eb : evecs;
    if (cur == eb && eb == ea) throw Error(NSP_ERR_ARG, "eig_restart: workspace aliasing");
    gemm_batched(c, m1, m, m1, ea, m1, 0, wl, m1, 0, cur, K, 0, 1);
    gemm_batched(c, m2, m, m2, tl_vec, m2p, 0, wr, m2, 0, cur + m1, K, 0, 1);
    double* lcur = lf;
    double* lother = la;
    for (int i = 1; i < d; ++i) {
      k_zvec<<<dim3(nb(m, 256), 1), 256, 0, c->stream>>>(m, m1, d, i, cur, 0, K, pm, sv, qm, 0, 0, zb, rho);
      NSP_HIP(hipGetLastError());
      secular<false>(c, sec, S, 1, m, lcur, 0, zb, 1, 0, rho, norm_t, bound, lother, 0, pos, 0, wbuf, 0, m);
      gemm_batched(c, m, m, m, cur, K, 0, wbuf, m, 0, other, K, 0, 1);
      std::swap(cur, other);
      std::swap(lcur, lother);
    }
    NSP_HIP(hipMemcpyAsync(evals, lcur, sizeof(double) * K, hipMemcpyDeviceToDevice, c->stream));
  }
}

EigWork* eig_work_new() { return new EigWork(); }
void eig_work_delete(EigWork* w) { delete w; }

}  // namespace nsp

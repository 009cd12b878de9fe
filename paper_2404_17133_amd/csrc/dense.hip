// Small dense FP64 solvers of the projected problems (Sec. 2.1: a = V^T A V is
// diagonalised; the linear-response and inner solves need shifted linear
// systems).  Sizes are the Krylov subspace dimension (tens to a few hundred),
// so each problem runs in one workgroup with the matrix in global memory
// (L2-resident); independent problems of a batch run in separate workgroups.
//
// small_eigh: cyclic Jacobi with the round-robin parallel ordering.  Every
// round pairs all indices into m/2 disjoint (p, q) pairs (index 0 fixed, the
// others rotated), computes the m/2 annihilating rotations from the current
// matrix, applies them to the rows, then to the columns and to the
// eigenvector matrix; disjoint rotations commute, so each phase is fully
// parallel.  A pair is rotated only while |a_pq| exceeds both
// 1e-15 sqrt(|a_pp a_qq|) (the classical threshold rule) and 4e-16 ||a||_F
// (the rounding level of the entries, so that rounding residue never
// re-triggers rotations); the sweeps stop after a sweep in which no pair
// needed a rotation (at most 40 sweeps).
#include <algorithm>

#include "engkern.hpp"

namespace rid {
namespace {

constexpr int DB = 1024;   // threads per dense workgroup
constexpr int MAXM = 1024; // largest projected dimension

__device__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  const int nw = blockDim.x >> 6;
  for (int w = 0; w < nw; ++w) s += red[w];
  return s;
}

// work: m*m + m doubles
__global__ __launch_bounds__(DB) void jacobi_kernel(double* a, int m, int lda, double* w, double* q, double* work) {
  __shared__ double cs[MAXM / 2], sn[MAXM / 2];
  __shared__ int pp[MAXM / 2], qq[MAXM / 2];
  __shared__ int rank[MAXM];
  __shared__ int nrot;
  __shared__ double red[16];
  const int tid = threadIdx.x;
  double fro = 0.0;
  for (int t = tid; t < m * m; t += DB) {
    q[t] = (t / m == t % m) ? 1.0 : 0.0;
    const double v = a[(long)(t / m) * lda + t % m];
    fro += v * v;
  }
  fro = sqrt(block_sum(fro, red));
  const double floor_abs = 4e-16 * fro;  // rounding level of the matrix entries
  const int mm = m + (m & 1);
  const int npair = mm / 2;
  __syncthreads();
  for (int sweep = 0; sweep < 40 && m > 1; ++sweep) {
    if (tid == 0) nrot = 0;
    __syncthreads();
    for (int r = 0; r < mm - 1; ++r) {
      if (tid < npair) {
        // round-robin slots: slot 0 fixed, slots 1..mm-1 shifted by r
        const int s1 = tid, s2 = mm - 1 - tid;
        int p = s1 == 0 ? 0 : 1 + (s1 - 1 + r) % (mm - 1);
        int qv = s2 == 0 ? 0 : 1 + (s2 - 1 + r) % (mm - 1);
        if (p > qv) {
          const int t = p;
          p = qv;
          qv = t;
        }
        double c = 1.0, s = 0.0;
        if (qv < m) {
          const double apq = a[(long)p * lda + qv];
          const double app = a[(long)p * lda + p], aqq = a[(long)qv * lda + qv];
          // rotate only while the coupling is above rounding level relative
          // to the two diagonal entries (the classical cyclic-Jacobi rule)
          if (fabs(apq) > 1e-15 * sqrt(fabs(app) * fabs(aqq)) && fabs(apq) > floor_abs) {
            const double tau = (aqq - app) / (2.0 * apq);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
            atomicAdd(&nrot, 1);
          }
        }
        pp[tid] = p;
        qq[tid] = qv;
        cs[tid] = c;
        sn[tid] = s;
      }
      __syncthreads();
      // rows: row_p' = c row_p - s row_q, row_q' = s row_p + c row_q
      for (int t = tid; t < npair * m; t += DB) {
        const int k = t / m, col = t - k * m;
        if (sn[k] == 0.0) continue;
        const int p = pp[k], qv = qq[k];
        const double c = cs[k], s = sn[k];
        const double x = a[(long)p * lda + col], y = a[(long)qv * lda + col];
        a[(long)p * lda + col] = c * x - s * y;
        a[(long)qv * lda + col] = s * x + c * y;
      }
      __syncthreads();
      // columns of a and of q
      for (int t = tid; t < npair * m; t += DB) {
        const int k = t / m, row = t - k * m;
        if (sn[k] == 0.0) continue;
        const int p = pp[k], qv = qq[k];
        const double c = cs[k], s = sn[k];
        double x = a[(long)row * lda + p], y = a[(long)row * lda + qv];
        a[(long)row * lda + p] = c * x - s * y;
        a[(long)row * lda + qv] = s * x + c * y;
        x = q[(long)row * m + p];
        y = q[(long)row * m + qv];
        q[(long)row * m + p] = c * x - s * y;
        q[(long)row * m + qv] = s * x + c * y;
      }
      __syncthreads();
    }
    const bool done = nrot == 0;
    __syncthreads();  // every thread has read nrot before it is reset
    if (done) break;
  }
  // ascending order, ties by index
  double* wd = work + (long)m * m;
  for (int i = tid; i < m; i += DB) wd[i] = a[(long)i * lda + i];
  __syncthreads();
  for (int i = tid; i < m; i += DB) {
    const double wi = wd[i];
    int r = 0;
    for (int j = 0; j < m; ++j) {
      const double wj = wd[j];
      r += (wj < wi) || (wj == wi && j < i);
    }
    rank[i] = r;
  }
  __syncthreads();
  for (int t = tid; t < m * m; t += DB) {
    const int i = t / m, j = t - i * m;
    work[(long)i * m + rank[j]] = q[t];
  }
  for (int j = tid; j < m; j += DB) w[rank[j]] = wd[j];
  __syncthreads();
  for (int t = tid; t < m * m; t += DB) q[t] = work[t];
}

// k lowest eigenpairs of a symmetric matrix: Householder reduction to
// tridiagonal form T = H^T a H (H = H_0 ... H_{m-3}), Sturm-count
// multisection (bisection with 64 points per step) for the eigenvalues of T,
// inverse iteration with partial pivoting for its eigenvectors
// (re-orthogonalised within clusters of close eigenvalues at every
// iteration), and back-transformation by the reflectors.
// work: 3 m + 6 m k + 2 m doubles.
__device__ inline int sturm_count(const double* __restrict__ d, const double* __restrict__ e2, int m, double x,
                                  double pivmin) {
  int cnt = 0;
  double qv = d[0] - x;
  if (fabs(qv) < pivmin) qv = -pivmin;
  cnt += qv < 0.0;
  for (int i = 1; i < m; ++i) {
    qv = d[i] - x - e2[i - 1] / qv;
    if (fabs(qv) < pivmin) qv = -pivmin;
    cnt += qv < 0.0;
  }
  return cnt;
}

constexpr int SYEVX_YLDS = 8192;  // inverse-iteration vectors held in LDS up to k * m = 8192

__global__ __launch_bounds__(DB) void syevx_kernel(double* a, int m, int lda, int k, double* w, double* q, int ldq,
                                                   double* work) {
  __shared__ double v[MAXM];
  __shared__ double wv[MAXM];
  __shared__ double pv[MAXM];  // pending update (absolute index)
  __shared__ double pw[MAXM];
  __shared__ double part[DB];
  __shared__ double red[16];
  __shared__ double sc[4];
  __shared__ double ylds[SYEVX_YLDS];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double* d = work;
  double* e = work + m;
  // work[2m, 3m) is unused (kept so the layout stays put)
  // k vectors of length m, in LDS when they fit (the work slot is then unused)
  double* y = (long)k * m <= SYEVX_YLDS ? ylds : work + 3 * m;
  double* fu = work + 3 * m + (long)k * m;  // factors u, s1, s2, l, piv: entry i of vector t at [i * k + t]
  double* fs1 = fu + (long)k * m;
  double* fs2 = fs1 + (long)k * m;
  double* fl = fs2 + (long)k * m;
  double* fp = fl + (long)k * m;
  int* refl = reinterpret_cast<int*>(fp + (long)k * m);  // reflector present flags (m ints)

  // ---- 1. tridiagonalisation ------------------------------------------------
  // Step j reflects column j below the diagonal (v) and would update the
  // trailing block A_t -= 2 (v w^T + w v^T), w = A_t v - (v^T A_t v) v.
  // That update is deferred: its vectors are kept (pv, pw, by absolute
  // index, zero where no update is pending) and applied on the fly where
  // the next step reads, so each step makes one pass over the trailing block
  // (apply the pending update, store, accumulate A_t v) instead of two.  The
  // stored values are the same expressions as an immediate update's, so the
  // result does not change.
  for (int i = tid; i < m; i += DB) {
    pv[i] = 0.0;
    pw[i] = 0.0;
  }
  __syncthreads();
  for (int j = 0; j + 2 < m; ++j) {
    const int n1 = m - j - 1;
    double ss = 0.0;
    for (int r = tid; r < n1; r += DB) {
      const int R = j + 1 + r;
      const double x = a[(long)R * lda + j] - 2.0 * (pv[R] * pw[j] + pw[R] * pv[j]);
      v[r] = x;
      ss += x * x;
    }
    ss = block_sum(ss, red);  // includes a barrier after the writes to v
    const double x0 = v[0];
    const double tail = ss - x0 * x0;
    if (tid == 0) d[j] = a[(long)j * lda + j] - 2.0 * (pv[j] * pw[j] + pw[j] * pv[j]);
    if (tail <= 1e-300 * (1.0 + ss)) {
      // column already reduced: no reflector (the pending update stays)
      if (tid == 0) {
        e[j] = x0;
        refl[j] = 0;
      }
      __syncthreads();
      continue;
    }
    const double sigma = sqrt(ss);
    const double alpha = x0 >= 0.0 ? -sigma : sigma;
    const double vn = sqrt(tail + (x0 - alpha) * (x0 - alpha));
    __syncthreads();
    for (int r = tid; r < n1; r += DB) {
      const double vr = (r == 0 ? x0 - alpha : v[r]) / vn;
      v[r] = vr;
      a[(long)j * lda + j + 1 + r] = vr;  // reflector kept in row j above the diagonal (unused from here on)
    }
    if (tid == 0) {
      e[j] = alpha;
      refl[j] = 1;
    }
    __syncthreads();
    // one pass over A_t: apply the pending update, store, and form the
    // column sums of A_t v (A_t symmetric), rows split in rg groups
    const int cw = ((n1 + 63) / 64) * 64;
    const int rg = max(1, DB / cw);
    {
      const int c = tid % cw, g = tid / cw;
      if (g < rg) {
        double acc = 0.0;
        if (c < n1) {
          const int C = j + 1 + c;
          const double pvc = pv[C], pwc = pw[C];
          for (int r = g; r < n1; r += rg) {
            const int R = j + 1 + r;
            double* ap = a + (long)R * lda + C;
            const double val = *ap - 2.0 * (pv[R] * pwc + pw[R] * pvc);
            *ap = val;
            acc += val * v[r];
          }
        }
        part[g * cw + c] = acc;
      }
    }
    __syncthreads();
    double kp = 0.0;
    for (int c = tid; c < n1; c += DB) {
      double pc = 0.0;
      for (int g = 0; g < rg; ++g) pc += part[g * cw + c];
      wv[c] = pc;
      kp += pc * v[c];
    }
    kp = block_sum(kp, red);  // barrier: wv complete
    // this step's update becomes the pending one
    for (int c = tid; c < n1; c += DB) {
      pv[j + 1 + c] = v[c];
      pw[j + 1 + c] = wv[c] - kp * v[c];
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (m >= 2) {
      d[m - 2] = a[(long)(m - 2) * lda + (m - 2)] - 2.0 * (pv[m - 2] * pw[m - 2] + pw[m - 2] * pv[m - 2]);
      e[m - 2] = a[(long)(m - 1) * lda + (m - 2)] - 2.0 * (pv[m - 1] * pw[m - 2] + pw[m - 1] * pv[m - 2]);
      if (m - 2 >= 0) refl[m - 2] = 0;
    }
    d[m - 1] = a[(long)(m - 1) * lda + (m - 1)] - 2.0 * (pv[m - 1] * pw[m - 1] + pw[m - 1] * pv[m - 1]);
    e[m - 1] = 0.0;
    refl[m - 1] = 0;
  }
  __syncthreads();  // d, e and refl are read by every thread below
  // ---- 2. eigenvalues of T by multisection ----------------------------------
  // Wave t brackets eigenvalue t (and t + 16, ...): its 64 lanes take Sturm
  // counts at 64 interior points of the bracket, which shrinks it 65-fold per
  // step, until its width is at the rounding level of the eigenvalue or of
  // ||T|| (the accuracy the counts support).  d and e^2 are staged in LDS.
  double tn = 0.0;
  for (int i = tid; i < m; i += DB) {
    v[i] = d[i];
    wv[i] = e[i] * e[i];
    tn = fmax(tn, fabs(d[i]) + fabs(e[i]) + (i > 0 ? fabs(e[i - 1]) : 0.0));
  }
  for (int o = 32; o > 0; o >>= 1) tn = fmax(tn, __shfl_xor(tn, o, 64));
  __syncthreads();
  if (lane == 0) red[wave] = tn;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int i = 0; i < DB / 64; ++i) t = fmax(t, red[i]);
    sc[0] = t;
  }
  __syncthreads();
  const double tnorm = fmax(sc[0], 1e-300);
  const double pivmin = 1e-300 + 1e-30 * tnorm * tnorm;
  const double atol = 2.2e-16 * tnorm;
  for (int t = wave; t < k; t += DB / 64) {
    double lo = -tnorm, hi = tnorm;
    for (int it = 0; it < 64; ++it) {
      const double wid = hi - lo;
      if (wid <= 2.2e-16 * fmax(fabs(lo), fabs(hi)) + atol) break;
      const double x = lo + wid * (double)(lane + 1) / 65.0;
      const unsigned long long above = __ballot(sturm_count(v, wv, m, x, pivmin) > t);
      if (above == 0ull) {
        lo = lo + wid * 64.0 / 65.0;
      } else {
        const int f = __ffsll(above) - 1;  // first point above eigenvalue t
        const double nlo = f > 0 ? lo + wid * (double)f / 65.0 : lo;
        hi = lo + wid * (double)(f + 1) / 65.0;
        lo = nlo;
      }
    }
    if (lane == 0) w[t] = 0.5 * (lo + hi);
  }
  __syncthreads();
  // ---- 3. inverse iteration ---------------------------------------------------
  // factor T - lambda_t I with partial pivoting (thread t), rows i, i+1 swapped
  // when |e_i| > |u_i|; u diagonal, s1/s2 the two superdiagonals, l multipliers.
  // The factors of the k shifts are interleaved (entry i of all shifts
  // adjacent), so the threads' loads are contiguous.
  if (tid < k) {
    const double lam = w[tid];
    const double eps_piv = 2.2e-16 * tnorm;
    double di = d[0] - lam, ci = m > 1 ? e[0] : 0.0;  // current row: diag, super
    for (int i = 0; i < m - 1; ++i) {
      const long at = (long)i * k + tid;
      const double bi = e[i];                // subdiagonal below the current row
      const double dn = d[i + 1] - lam;       // next row diag
      const double cn = (i + 1 < m - 1) ? e[i + 1] : 0.0;  // next row super
      if (fabs(di) >= fabs(bi)) {
        // no swap: eliminate next row with the current one
        const double piv = fabs(di) < eps_piv ? (di < 0 ? -eps_piv : eps_piv) : di;
        const double mult = bi / piv;
        fu[at] = piv;
        fs1[at] = ci;
        fs2[at] = 0.0;
        fl[at] = mult;
        fp[at] = 0.0;
        di = dn - mult * ci;
        ci = cn;
      } else {
        // swap rows i and i+1
        const double mult = di / bi;
        fu[at] = bi;
        fs1[at] = dn;
        fs2[at] = cn;
        fl[at] = mult;
        fp[at] = 1.0;
        di = ci - mult * dn;
        ci = -mult * cn;
      }
    }
    fu[(long)(m - 1) * k + tid] = fabs(di) < eps_piv ? (di < 0 ? -eps_piv : eps_piv) : di;
    // starting vector: deterministic, not orthogonal to any eigenvector in practice
    double* yt = y + (long)tid * m;
    for (int i = 0; i < m; ++i) yt[i] = 1.0 + 0.01 * (double)((i * 7919 + tid * 104729) % 101) / 101.0;
  }
  __syncthreads();
  // clusters of close eigenvalues (consecutive gaps <= 1e-3 ||T||): cluster c
  // is handled by wave c mod 16, which orthogonalises its vectors in
  // ascending order; other waves never touch them, so no block barrier is
  // needed between vectors.
  const double gap = 1e-3 * tnorm;
  for (int iter = 0; iter < 4; ++iter) {
    if (tid < k) {
      double* yt = y + (long)tid * m;
      // forward: row interchanges and multipliers (y_i carried in yc)
      double yc = yt[0];
#pragma unroll 4
      for (int i = 0; i < m - 1; ++i) {
        const long at = (long)i * k + tid;
        const double yn = yt[i + 1];
        if (fp[at] != 0.0) {
          yt[i] = yn;
          yc = yc - fl[at] * yn;
        } else {
          yt[i] = yc;
          yc = yn - fl[at] * yc;
        }
      }
      yt[m - 1] = yc;
      // backward: upper triangular with two superdiagonals (y_{i+1}, y_{i+2}
      // carried in y1, y2)
      double y1 = 0.0, y2 = 0.0;
#pragma unroll 4
      for (int i = m - 1; i >= 0; --i) {
        const long at = (long)i * k + tid;
        double t = yt[i];
        if (i + 1 < m) t -= fs1[at] * y1;
        if (i + 2 < m) t -= fs2[at] * y2;
        const double yi = t / fu[at];
        yt[i] = yi;
        y2 = y1;
        y1 = yi;
      }
    }
    __syncthreads();
    int cl = -1;
    for (int t = 0; t < k; ++t) {
      if (t == 0 || fabs(w[t - 1] - w[t]) > gap) ++cl;  // t starts cluster cl
      if (cl % (DB / 64) != wave) continue;
      int t0 = t;
      while (t0 > 0 && fabs(w[t0 - 1] - w[t0]) <= gap) --t0;
      double* yt = y + (long)t * m;
      for (int s2 = t0; s2 < t; ++s2) {
        const double* ys = y + (long)s2 * m;
        double dp = 0.0;
        for (int i = lane; i < m; i += 64) dp += ys[i] * yt[i];
        dp = wave_sum(dp);
        for (int i = lane; i < m; i += 64) yt[i] -= dp * ys[i];
      }
      double nn = 0.0;
      for (int i = lane; i < m; i += 64) nn += yt[i] * yt[i];
      nn = wave_sum(nn);
      const double inv = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
      for (int i = lane; i < m; i += 64) yt[i] *= inv;
    }
    __syncthreads();
  }
  // ---- 4. back-transformation, one wave per vector ----------------------------
  // y <- H_0 ... H_{m-3} y with the vector in registers (entry i in lane
  // i % 64, slot i / 64); reflector j is row j of a right of the diagonal.
  for (int t = wave; t < k; t += DB / 64) {
    double* yt = y + (long)t * m;
    double yr[MAXM / 64];
#pragma unroll
    for (int sl = 0; sl < MAXM / 64; ++sl) {
      const int i = sl * 64 + lane;
      yr[sl] = i < m ? yt[i] : 0.0;
    }
    for (int j = m - 3; j >= 0; --j) {
      if (!refl[j]) continue;
      const double* hrow = a + (long)j * lda;
      double h[MAXM / 64];
      double dp = 0.0;
#pragma unroll
      for (int sl = 0; sl < MAXM / 64; ++sl) {
        const int i = sl * 64 + lane;
        h[sl] = (i > j && i < m) ? hrow[i] : 0.0;
        dp += h[sl] * yr[sl];
      }
      dp = wave_sum(dp);
#pragma unroll
      for (int sl = 0; sl < MAXM / 64; ++sl) yr[sl] -= 2.0 * dp * h[sl];
    }
#pragma unroll
    for (int sl = 0; sl < MAXM / 64; ++sl) {
      const int i = sl * 64 + lane;
      if (i < m) yt[i] = yr[sl];
    }
  }
  __syncthreads();
  for (long idx = tid; idx < (long)m * k; idx += DB) {
    const int i = (int)(idx / k), t = (int)(idx - (long)i * k);
    q[(long)i * ldq + t] = y[(long)t * m + i];
  }
}

// Cholesky, left-looking by columns.
// Cholesky of a small matrix (m <= 64) by one wavefront in LDS, right
// looking: lane i owns row i.  Same contract as chol_kernel (lower factor in
// place, upper zeroed, info = first non-positive pivot + 1, such a pivot
// replaced by 1).  For the block Gram matrices of the orthonormalisation,
// where the 1024-thread kernel's per-column reductions dominate.
constexpr int CHOL_SMALL = 64;

__global__ __launch_bounds__(64) void chol_small_kernel(double* a, int m, int lda, int* info) {
  __shared__ double sa[CHOL_SMALL][CHOL_SMALL + 1];
  const int i = threadIdx.x;
  if (i < m)
    for (int k = 0; k <= i; ++k) sa[i][k] = a[(long)i * lda + k];
  int bad = 0;
  __syncthreads();
  for (int j = 0; j < m; ++j) {
    const double d = sa[j][j];
    if (!(d > 0.0) && !bad) bad = j + 1;
    const double piv = d > 0.0 ? sqrt(d) : 1.0;
    __syncthreads();  // every lane has read the pivot
    if (i == j) sa[j][j] = piv;
    if (i > j && i < m) sa[i][j] /= piv;
    __syncthreads();
    if (i > j && i < m) {
      const double li = sa[i][j];
      for (int k = j + 1; k <= i; ++k) sa[i][k] -= li * sa[k][j];
    }
    __syncthreads();
  }
  if (i < m)
    for (int k = 0; k < m; ++k) a[(long)i * lda + k] = k <= i ? sa[i][k] : 0.0;
  if (i == 0) info[0] = bad;
}

__global__ __launch_bounds__(DB) void chol_kernel(double* a, int m, int lda, int* info) {
  __shared__ double red[16];
  __shared__ double piv;
  __shared__ int bad;
  const int tid = threadIdx.x;
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int j = 0; j < m; ++j) {
    double s = 0.0;
    for (int k = tid; k < j; k += DB) s += a[(long)j * lda + k] * a[(long)j * lda + k];
    s = block_sum(s, red);
    if (tid == 0) {
      const double d = a[(long)j * lda + j] - s;
      if (!(d > 0.0) && !bad) bad = j + 1;
      piv = d > 0.0 ? sqrt(d) : 1.0;
      a[(long)j * lda + j] = piv;
    }
    __syncthreads();
    for (int i = j + 1 + tid; i < m; i += DB) {
      double t = a[(long)i * lda + j];
      for (int k = 0; k < j; ++k) t -= a[(long)i * lda + k] * a[(long)j * lda + k];
      a[(long)i * lda + j] = t / piv;
    }
    __syncthreads();
  }
  for (int t = tid; t < m * m; t += DB) {
    const int i = t / m, j = t - i * m;
    if (j > i) a[(long)i * lda + j] = 0.0;
  }
  if (tid == 0) info[0] = bad;
}

// Cholesky by panels of NBC columns, right looking (64 < m <= 512).  The
// panel (its rows j0..m-1) is factored column by column in LDS, written
// back, and then applied to the trailing lower triangle as one rank-NBC
// update: lanes run along a row of the trailing block (coalesced), each
// holding the panel entries of its own column in registers, and the panel
// row of the output row is read by all lanes at once.  Every trailing
// element is read and written once per panel; the column-wise kernel above
// instead walks each row in a separate thread, with every load spread over
// 64 rows.  Same contract as chol_kernel.
constexpr int CHOL_BLK_MAX = 512;
constexpr int NBC = 16;

__global__ __launch_bounds__(DB) void chol_blocked_kernel(double* a, int m, int lda, int* info) {
  __shared__ double pan[CHOL_BLK_MAX * (NBC + 1)];  // pan[r * (NBC + 1) + c], row r counted from j0
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int bad = 0;  // meaningful in thread 0
  for (int j0 = 0; j0 < m; j0 += NBC) {
    const int nb = min(NBC, m - j0);
    const int rows = m - j0;
    // 1. panel to LDS (entries above the diagonal are loaded but never used)
    for (int e = tid; e < rows * nb; e += DB) {
      const int r = e / nb, c = e - r * nb;
      pan[r * (NBC + 1) + c] = a[(long)(j0 + r) * lda + j0 + c];
    }
    __syncthreads();
    // 2. factor the panel
    for (int c = 0; c < nb; ++c) {
      const double d = pan[c * (NBC + 1) + c];
      __syncthreads();  // every thread has read the pivot
      if (tid == 0 && !(d > 0.0) && !bad) bad = j0 + c + 1;
      const double piv = d > 0.0 ? sqrt(d) : 1.0;
      for (int r = c + tid; r < rows; r += DB) pan[r * (NBC + 1) + c] = r == c ? piv : pan[r * (NBC + 1) + c] / piv;
      __syncthreads();
      const int w = nb - c - 1;
      for (int e = tid; e < (rows - c - 1) * w; e += DB) {
        const int r = c + 1 + e / w, c2 = c + 1 + e % w;
        if (c2 <= r) pan[r * (NBC + 1) + c2] -= pan[r * (NBC + 1) + c] * pan[c2 * (NBC + 1) + c];
      }
      __syncthreads();
    }
    // 3. panel back to memory (lower part)
    for (int e = tid; e < rows * nb; e += DB) {
      const int r = e / nb, c = e - r * nb;
      if (c <= r) a[(long)(j0 + r) * lda + j0 + c] = pan[r * (NBC + 1) + c];
    }
    // 4. trailing update A22 -= L21 L21^T on the lower triangle.  A trailing
    // block exists only when this panel is full (nb == NBC).
    const int k1 = j0 + nb, mt = m - k1;
    if (mt > 0) {
      const int bands = (mt + 63) / 64;       // 64-column bands, at most 8
      const int rg = max(1, (DB / 64) / bands);  // waves per band, split over rows
      const int band = wave % bands, g = wave / bands;
      if (g < rg) {
        const int kc = band * 64 + lane;  // column in the trailing block
        double lk[NBC];
#pragma unroll
        for (int p = 0; p < NBC; ++p) lk[p] = kc < mt ? pan[(nb + kc) * (NBC + 1) + p] : 0.0;
        for (int i0 = band * 64 + g; i0 < mt; i0 += 4 * rg) {
          double av[4], t[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int i = i0 + u * rg;
            av[u] = (kc < mt && i < mt && kc <= i) ? a[(long)(k1 + i) * lda + k1 + kc] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int i = i0 + u * rg;
            double s = 0.0;
            if (i < mt) {
              const double* pr = pan + (nb + i) * (NBC + 1);
#pragma unroll
              for (int p = 0; p < NBC; ++p) s += pr[p] * lk[p];
            }
            t[u] = s;
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int i = i0 + u * rg;
            if (kc < mt && i < mt && kc <= i) a[(long)(k1 + i) * lda + k1 + kc] = av[u] - t[u];
          }
        }
      }
    }
    __syncthreads();
  }
  for (int t = tid; t < m * m; t += DB) {
    const int i = t / m, j = t - i * m;
    if (j > i) a[(long)i * lda + j] = 0.0;
  }
  if (tid == 0) info[0] = bad;
}

// Gaussian elimination with partial pivoting, one system per workgroup.
__global__ __launch_bounds__(DB) void lu_solve_kernel(double* mats, double* rhs, int m) {
  __shared__ double rv[16];
  __shared__ int ri[16];
  __shared__ int pivrow;
  __shared__ double pivval, yj;
  double* a = mats + (long)blockIdx.x * m * m;
  double* g = rhs + (long)blockIdx.x * m;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int j = 0; j < m; ++j) {
    // pivot: argmax |a[i][j]| over i >= j (ties to the smaller index)
    double best = -1.0;
    int bi = j;
    for (int i = j + tid; i < m; i += DB) {
      const double v = fabs(a[(long)i * m + j]);
      if (v > best) {
        best = v;
        bi = i;
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(best, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
      }
    }
    if (lane == 0) {
      rv[wave] = best;
      ri[wave] = bi;
    }
    __syncthreads();
    if (tid == 0) {
      double b = -1.0;
      int bidx = j;
      for (int w = 0; w < (DB >> 6); ++w)
        if (rv[w] > b || (rv[w] == b && ri[w] < bidx)) {
          b = rv[w];
          bidx = ri[w];
        }
      pivrow = bidx;
    }
    __syncthreads();
    const int pr = pivrow;
    if (pr != j) {
      for (int k = tid; k < m; k += DB) {
        const double t = a[(long)j * m + k];
        a[(long)j * m + k] = a[(long)pr * m + k];
        a[(long)pr * m + k] = t;
      }
      if (tid == 0) {
        const double t = g[j];
        g[j] = g[pr];
        g[pr] = t;
      }
    }
    __syncthreads();
    if (tid == 0) {
      double p = a[(long)j * m + j];
      if (fabs(p) < 1e-300) p = p < 0.0 ? -1e-300 : 1e-300;
      a[(long)j * m + j] = p;
      pivval = p;
    }
    __syncthreads();
    const double pv = pivval;
    // eliminate below: one row per thread group
    for (int i = j + 1 + tid; i < m; i += DB) {
      const double l = a[(long)i * m + j] / pv;
      a[(long)i * m + j] = l;
    }
    __syncthreads();
    const int rowsb = m - j - 1;
    for (int t = tid; t < rowsb * (m - j); t += DB) {
      const int i = j + 1 + t / (m - j);
      const int k = j + t % (m - j);
      if (k == j) {
        g[i] -= a[(long)i * m + j] * g[j];
      } else {
        a[(long)i * m + k] -= a[(long)i * m + j] * a[(long)j * m + k];
      }
    }
    __syncthreads();
  }
  // back substitution by columns
  for (int j = m - 1; j >= 0; --j) {
    if (tid == 0) {
      yj = g[j] / a[(long)j * m + j];
      g[j] = yj;
    }
    __syncthreads();
    const double y = yj;
    for (int i = tid; i < j; i += DB) g[i] -= a[(long)i * m + j] * y;
    __syncthreads();
  }
}

// Gaussian elimination with partial pivoting on column-major systems
// (a(i, k) at a[k m + i]), one system per workgroup of LB threads.  Thread t
// owns rows t, t + LB, ...: it computes their multipliers and updates them,
// reading the pivot row by broadcast and its own rows with coalesced
// accesses, so that a column needs two barriers (pivot choice, row swap).
// The pivot search of column j + 1 visits exactly the rows each thread
// updated at column j, so no barrier separates the two.
constexpr int LB = 256;
constexpr int LU_MAX = 2048;  // largest system of lu_cm_kernel (pivot row staged in LDS)

__device__ inline double guard_pivot(double p) { return fabs(p) < 1e-300 ? (p < 0.0 ? -1e-300 : 1e-300) : p; }

__global__ __launch_bounds__(LB) void lu_cm_kernel(double* mats, double* rhs, int m) {
  __shared__ double rv[LB / 64];
  __shared__ int ri[LB / 64];
  __shared__ double prow[LU_MAX];
  double* a = mats + (long)blockIdx.x * m * m;
  double* g = rhs + (long)blockIdx.x * m;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int j = 0; j < m; ++j) {
    // pivot: argmax |a(i, j)| over i >= j (ties to the smaller index)
    double best = -1.0;
    int bi = m;
    for (int i = j + tid; i < m; i += LB) {
      const double v = fabs(a[(long)j * m + i]);
      if (v > best) {
        best = v;
        bi = i;
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(best, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
      }
    }
    if (lane == 0) {
      rv[wave] = best;
      ri[wave] = bi;
    }
    __syncthreads();
    double pb = -1.0;
    int p = j;
    for (int w = 0; w < LB / 64; ++w)
      if (rv[w] > pb || (rv[w] == pb && ri[w] < p)) {
        pb = rv[w];
        p = ri[w];
      }
    if (p >= m) p = j;
    if (p != j) {
      for (int k = tid; k < m; k += LB) {
        const double t = a[(long)k * m + j];
        a[(long)k * m + j] = a[(long)k * m + p];
        a[(long)k * m + p] = t;
      }
      if (tid == 0) {
        const double t = g[j];
        g[j] = g[p];
        g[p] = t;
      }
    }
    __syncthreads();
    // the pivot row right of the diagonal, staged in LDS once for all rows
    // (read from memory for systems larger than the staging buffer)
    const bool staged = m <= LU_MAX;
    if (staged)
      for (int k = j + 1 + tid; k < m; k += LB) prow[k] = a[(long)k * m + j];
    const double pv = guard_pivot(a[(long)j * m + j]);
    const double gj = g[j];
    __syncthreads();
    for (int i = j + 1 + tid; i < m; i += LB) {
      const double l = a[(long)j * m + i] / pv;
      a[(long)j * m + i] = l;
      // eight independent loads in flight per step of the row update
      int k = j + 1;
      for (; k + 8 <= m; k += 8) {
        double v[8], u[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          v[q] = a[(long)(k + q) * m + i];
          u[q] = staged ? prow[k + q] : a[(long)(k + q) * m + j];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) a[(long)(k + q) * m + i] = v[q] - l * u[q];
      }
      for (; k < m; ++k) a[(long)k * m + i] -= l * (staged ? prow[k] : a[(long)k * m + j]);
      g[i] -= l * gj;
    }
  }
  // back substitution with U (diagonal guarded as in the elimination)
  for (int j = m - 1; j >= 0; --j) {
    __syncthreads();
    const double yj = g[j] / guard_pivot(a[(long)j * m + j]);
    __syncthreads();
    if (tid == 0) g[j] = yj;
    for (int i = tid; i < j; i += LB) g[i] -= a[(long)j * m + i] * yj;
  }
}

// The same elimination for systems small enough to live in LDS (m <= 128:
// 132 KB with an odd leading dimension): the matrix and the right-hand side
// are copied in once, every column step works on LDS only, with the trailing
// update spread over all threads of the block (not one row per thread), and
// only the solution is written back.  Pivot choice, guard and operation
// order per element are those of lu_cm_kernel.
constexpr int LU_LDS_MAX = 128;

__global__ __launch_bounds__(LB) void lu_lds_kernel(const double* mats, double* rhs, int m) {
  __shared__ double sa[LU_LDS_MAX * (LU_LDS_MAX + 1)];
  __shared__ double sg[LU_LDS_MAX];
  __shared__ double rv[LB / 64];
  __shared__ int ri[LB / 64];
  const int ld = m | 1;  // odd: the row swap's strided accesses spread over the banks
  const double* a = mats + (long)blockIdx.x * m * m;
  double* g = rhs + (long)blockIdx.x * m;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int e = tid; e < m * m; e += LB) {
    const int k = e / m, i = e - k * m;
    sa[k * ld + i] = a[e];
  }
  for (int i = tid; i < m; i += LB) sg[i] = g[i];
  __syncthreads();
  for (int j = 0; j < m; ++j) {
    double best = -1.0;
    int bi = m;
    for (int i = j + tid; i < m; i += LB) {
      const double v = fabs(sa[j * ld + i]);
      if (v > best) {
        best = v;
        bi = i;
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(best, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
      }
    }
    if (lane == 0) {
      rv[wave] = best;
      ri[wave] = bi;
    }
    __syncthreads();
    double pb = -1.0;
    int p = j;
    for (int w = 0; w < LB / 64; ++w)
      if (rv[w] > pb || (rv[w] == pb && ri[w] < p)) {
        pb = rv[w];
        p = ri[w];
      }
    if (p >= m) p = j;
    if (p != j) {
      for (int k = tid; k < m; k += LB) {
        const double t = sa[k * ld + j];
        sa[k * ld + j] = sa[k * ld + p];
        sa[k * ld + p] = t;
      }
      if (tid == 0) {
        const double t = sg[j];
        sg[j] = sg[p];
        sg[p] = t;
      }
    }
    __syncthreads();
    // multipliers of column j and the right-hand side
    const double pv = guard_pivot(sa[j * ld + j]);
    const double gj = sg[j];
    for (int i = j + 1 + tid; i < m; i += LB) {
      const double l = sa[j * ld + i] / pv;
      sa[j * ld + i] = l;
      sg[i] -= l * gj;
    }
    __syncthreads();
    // trailing update, element (i, k) of the (m-j-1)^2 block per thread
    // (linear index e = kk r + ii stepped without a division per element)
    const int r = m - j - 1;
    if (r > 0) {
      const int dk = LB / r, di = LB - dk * r;
      int kk = tid / r, ii = tid - kk * r;
      for (int e = tid; e < r * r; e += LB) {
        const int i = j + 1 + ii, k = j + 1 + kk;
        sa[k * ld + i] -= sa[j * ld + i] * sa[k * ld + j];
        ii += di;
        kk += dk;
        if (ii >= r) {
          ii -= r;
          ++kk;
        }
      }
    }
    __syncthreads();
  }
  for (int j = m - 1; j >= 0; --j) {
    const double yj = sg[j] / guard_pivot(sa[j * ld + j]);
    __syncthreads();
    if (tid == 0) sg[j] = yj;
    for (int i = tid; i < j; i += LB) sg[i] -= sa[j * ld + i] * yj;
    __syncthreads();
  }
  for (int i = tid; i < m; i += LB) g[i] = sg[i];
}

// Blocked right-looking elimination for 128 < m <= LU_BLK_MAX (matrix in
// global memory, column-major, destroyed).  Per panel of NBK columns: the
// panel (rows j0..m) is factored in LDS with the same partial pivoting as
// lu_cm_kernel, the right-hand side (kept in LDS) is eliminated alongside,
// the panel's row swaps are applied to the trailing columns, the panel rows
// of the trailing columns are solved with the unit lower factor (U12, also
// staged in LDS), and the trailing block takes one rank-NBK update spread
// over all threads.  Every trailing element is read and written once per
// panel instead of once per column.
constexpr int LU_BLK_MAX = 512;
constexpr int NBK = 16;

__device__ inline void block_argmax(double v, int idx, double* rv, int* ri, double& best, int& bi) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_xor(v, o, 64);
    const int oi = __shfl_xor(idx, o, 64);
    if (ov > v || (ov == v && oi < idx)) {
      v = ov;
      idx = oi;
    }
  }
  if (lane == 0) {
    rv[wave] = v;
    ri[wave] = idx;
  }
  __syncthreads();
  best = -1.0;
  bi = 1 << 30;
  for (int w = 0; w < LB / 64; ++w)
    if (rv[w] > best || (rv[w] == best && ri[w] < bi)) {
      best = rv[w];
      bi = ri[w];
    }
}

__global__ __launch_bounds__(LB) void lu_blocked_kernel(double* mats, double* rhs, int m) {
  __shared__ double pan[NBK * LU_BLK_MAX];  // panel: pan[c * m + r], rows r >= j0 used
  __shared__ double u12[NBK * LU_BLK_MAX];  // panel rows of the trailing columns: u12[c * m + k]
  __shared__ double sg[LU_BLK_MAX];
  __shared__ int piv[NBK];
  __shared__ double rv[LB / 64];
  __shared__ int ri[LB / 64];
  double* a = mats + (long)blockIdx.x * m * m;
  double* g = rhs + (long)blockIdx.x * m;
  const int tid = threadIdx.x;
  for (int i = tid; i < m; i += LB) sg[i] = g[i];
  for (int j0 = 0; j0 < m; j0 += NBK) {
    const int nb = min(NBK, m - j0);
    const int k1 = j0 + nb;  // first trailing column
    // 1. panel to LDS
    for (int e = tid; e < nb * (m - j0); e += LB) {
      const int c = e / (m - j0), r = j0 + e % (m - j0);
      pan[c * m + r] = a[(long)(j0 + c) * m + r];
    }
    __syncthreads();
    // 2. factor the panel (and eliminate the right-hand side)
    for (int c = 0; c < nb; ++c) {
      const int j = j0 + c;
      double v = -1.0;
      int idx = 1 << 30;
      for (int i = j + tid; i < m; i += LB) {
        const double t = fabs(pan[c * m + i]);
        if (t > v) {
          v = t;
          idx = i;
        }
      }
      double best;
      int p;
      block_argmax(v, idx, rv, ri, best, p);
      if (p >= m) p = j;
      if (tid == 0) piv[c] = p;
      if (p != j) {
        for (int cc = tid; cc < nb; cc += LB) {
          const double t = pan[cc * m + j];
          pan[cc * m + j] = pan[cc * m + p];
          pan[cc * m + p] = t;
        }
        if (tid == 0) {
          const double t = sg[j];
          sg[j] = sg[p];
          sg[p] = t;
        }
      }
      __syncthreads();
      const double pv = guard_pivot(pan[c * m + j]);
      const double gj = sg[j];
      for (int i = j + 1 + tid; i < m; i += LB) {
        const double l = pan[c * m + i] / pv;
        pan[c * m + i] = l;
        sg[i] -= l * gj;
      }
      __syncthreads();
      // rest of the panel: columns c + 1 .. nb - 1
      const int r = m - j - 1;
      if (r > 0) {
        const int dk = LB / r, di = LB - dk * r;
        int kk = tid / r, ii = tid - kk * r;
        for (int e = tid; e < r * (nb - c - 1); e += LB) {
          const int cc = c + 1 + kk, i = j + 1 + ii;
          pan[cc * m + i] -= pan[c * m + i] * pan[cc * m + j];
          ii += di;
          kk += dk;
          if (ii >= r) {
            ii -= r;
            ++kk;
          }
        }
      }
      __syncthreads();
    }
    // 3. panel back to memory
    for (int e = tid; e < nb * (m - j0); e += LB) {
      const int c = e / (m - j0), r = j0 + e % (m - j0);
      a[(long)(j0 + c) * m + r] = pan[c * m + r];
    }
    if (k1 < m) {
      // 4. the panel's row swaps on the trailing columns, in order
      for (int k = k1 + tid; k < m; k += LB) {
        double* col = a + (long)k * m;
        for (int c = 0; c < nb; ++c) {
          const int p = piv[c];
          if (p != j0 + c) {
            const double t = col[j0 + c];
            col[j0 + c] = col[p];
            col[p] = t;
          }
        }
        // 5. U12 = L11^{-1} A12 for this column (unit lower triangular)
        double u[NBK];
#pragma unroll
        for (int c = 0; c < NBK; ++c) {
          if (c < nb) {
            double t = col[j0 + c];
            for (int cp = 0; cp < c; ++cp) t -= pan[cp * m + j0 + c] * u[cp];
            u[c] = t;
            col[j0 + c] = t;
            u12[c * m + k] = t;
          }
        }
      }
      __syncthreads();
      // 6. trailing update A22 -= L21 U12
      // (linear index e = kk r + ii stepped without a division per element)
      const int r = m - k1, w = m - k1;
      const int dk = LB / r, di = LB - dk * r;
      int kk = tid / r, ii = tid - kk * r;
      for (int e = tid; e < r * w; e += LB) {
        const int i = k1 + ii, k = k1 + kk;
        double t = a[(long)k * m + i];
        // a trailing block exists only below a full panel (nb == NBK)
#pragma unroll
        for (int c = 0; c < NBK; ++c) t -= pan[c * m + i] * u12[c * m + k];
        a[(long)k * m + i] = t;
        ii += di;
        kk += dk;
        if (ii >= r) {
          ii -= r;
          ++kk;
        }
      }
    }
    __syncthreads();
  }
  // back substitution with U by blocks of NBK rows from the bottom: the
  // diagonal block is staged in LDS and solved by one thread, then every
  // thread subtracts the block's columns from its rows above.  Each row
  // receives its subtractions in the same order (descending columns) as
  // the column-at-a-time substitution, so the result is bit-identical.
  for (int j1 = m; j1 > 0; j1 -= NBK) {
    const int jb = max(0, j1 - NBK), nb = j1 - jb;
    for (int e = tid; e < nb * nb; e += LB) {
      const int c = e / nb, r = e - c * nb;
      pan[c * (NBK + 1) + r] = a[(long)(jb + c) * m + jb + r];
    }
    __syncthreads();
    if (tid == 0) {
      for (int r = nb - 1; r >= 0; --r) {
        double t = sg[jb + r];
        for (int c = nb - 1; c > r; --c) t -= pan[c * (NBK + 1) + r] * sg[jb + c];
        sg[jb + r] = t / guard_pivot(pan[r * (NBK + 1) + r]);
      }
    }
    __syncthreads();
    for (int i = tid; i < jb; i += LB) {
      double t = sg[i];
      for (int c = nb - 1; c >= 0; --c) t -= a[(long)(jb + c) * m + i] * sg[jb + c];
      sg[i] = t;
    }
    __syncthreads();
  }
  for (int i = tid; i < m; i += LB) g[i] = sg[i];
}

// Pair systems of the inner full-TDDFT solve.  System q of right-hand side
// b = sys_b[q]: type 0 (shift s != 0): (t- t+ - s^2 I) y = t- g1 + s g2;
// type 1 (s = 0): t+ y = g1; type 2 (s = 0): t- y' = g2.  Matrices are
// written column-major for lu_cm_kernel.
__global__ void pair_mats_kernel(const double* __restrict__ P, const double* __restrict__ tp,
                                 const double* __restrict__ tm, int ld, int m, const int* __restrict__ sys_type,
                                 const double* __restrict__ sys_shift, double* __restrict__ mats) {
  const int q = blockIdx.y;
  const int type = sys_type[q];
  const double s2 = sys_shift[q] * sys_shift[q];
  double* out = mats + (long)q * m * m;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < m * m; e += gridDim.x * blockDim.x) {
    const int k = e / m, i = e - k * m;  // out(i, k) at k m + i
    double v;
    if (type == 0)
      v = P[(long)i * m + k] - (i == k ? s2 : 0.0);
    else if (type == 1)
      v = tp[(long)i * ld + k];
    else
      v = tm[(long)i * ld + k];
    out[e] = v;
  }
}

__global__ void pair_rhs_kernel(const double* __restrict__ g, int ldg, const double* __restrict__ tg,
                                const int* __restrict__ sys_b, const int* __restrict__ sys_type,
                                const double* __restrict__ sys_shift, int nsys, int m, double* __restrict__ rhs) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nsys * m) return;
  const int q = t / m, i = t - q * m;
  const int b = sys_b[q], type = sys_type[q];
  const double* g1 = g + (long)b * ldg;
  const double* g2 = g1 + m;
  double v;
  if (type == 0)
    v = tg[(long)b * m + i] + sys_shift[q] * g2[i];
  else if (type == 1)
    v = g1[i];
  else
    v = g2[i];
  rhs[(long)q * m + i] = v;
}

// Write the solutions back: type 0 gives y and y' = (t+ y - g1) / s (yt =
// y t+), type 1 gives y, type 2 gives y'.
__global__ void pair_unpack_kernel(double* __restrict__ g, int ldg, const double* __restrict__ sol,
                                   const double* __restrict__ yt, const int* __restrict__ sys_b,
                                   const int* __restrict__ sys_type, const double* __restrict__ sys_shift, int nsys,
                                   int m) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nsys * m) return;
  const int q = t / m, i = t - q * m;
  const int b = sys_b[q], type = sys_type[q];
  double* g1 = g + (long)b * ldg;
  double* g2 = g1 + m;
  const double y = sol[(long)q * m + i];
  if (type == 0) {
    g2[i] = (yt[(long)q * m + i] - g1[i]) / sys_shift[q];
    g1[i] = y;
  } else if (type == 1) {
    g1[i] = y;
  } else {
    g2[i] = y;
  }
}

// Tiled small GEMM, 16x16 tiles.
__global__ void small_gemm_kernel(int ta, int tb, int m, int n, int k, double alpha, const double* __restrict__ A,
                                  int lda, const double* __restrict__ B, int ldb, double beta, double* C, int ldc) {
  __shared__ double As[16][17], Bs[16][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int row = blockIdx.y * 16 + ty, col = blockIdx.x * 16 + tx;
  double acc = 0.0;
  for (int k0 = 0; k0 < k; k0 += 16) {
    const int ka = k0 + tx, kb = k0 + ty;
    // As[ty][tx] = op(A)[row][ka]
    double av = 0.0;
    if (row < m && ka < k) av = ta ? A[(long)ka * lda + row] : A[(long)row * lda + ka];
    As[ty][tx] = av;
    double bv = 0.0;
    if (col < n && kb < k) bv = tb ? B[(long)col * ldb + kb] : B[(long)kb * ldb + col];
    Bs[ty][tx] = bv;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) acc += As[ty][q] * Bs[q][tx];
    __syncthreads();
  }
  if (row < m && col < n) {
    double* c = C + (long)row * ldc + col;
    *c = (beta == 0.0 ? 0.0 : beta * *c) + alpha * acc;
  }
}

// G = L^{-1} for lower-triangular L, one column per thread.
__global__ void trinv_lower_kernel(const double* __restrict__ L, int m, int ldl, double* __restrict__ G, int ldg) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= m) return;
  for (int i = 0; i < c; ++i) G[(long)i * ldg + c] = 0.0;
  G[(long)c * ldg + c] = 1.0 / L[(long)c * ldl + c];
  for (int i = c + 1; i < m; ++i) {
    double acc = 0.0;
    for (int k = c; k < i; ++k) acc += L[(long)i * ldl + k] * G[(long)k * ldg + c];
    G[(long)i * ldg + c] = -acc / L[(long)i * ldl + i];
  }
}

// mats_b = t - sh_b^2 w  (m x m each)
__global__ void build_schur_kernel(const double* __restrict__ t, int ldt, const double* __restrict__ w, int ldw, int m,
                                   const double* __restrict__ sh, double* __restrict__ mats) {
  const int b = blockIdx.y;
  const double s2 = sh[b] * sh[b];
  double* out = mats + (long)b * m * m;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < m * m; e += gridDim.x * blockDim.x) {
    const int i = e / m, j = e - i * m;
    out[e] = t[(long)i * ldt + j] - s2 * w[(long)i * ldw + j];
  }
}

// out_b = x_b + sh_b * y_b for rows b < nb of length m
__global__ void rows_axpy_kernel(const double* __restrict__ x, int ldx, const double* __restrict__ y, int ldy,
                                 const double* __restrict__ sh, int nb, int m, double* __restrict__ out, int ldo) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nb * m) return;
  const int b = t / m, i = t - b * m;
  out[(long)b * ldo + i] = x[(long)b * ldx + i] + sh[b] * y[(long)b * ldy + i];
}

__global__ void symmetrize_kernel(double* a, int m, int lda) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m * m) return;
  const int i = t / m, j = t - i * m;
  if (j <= i) return;
  const double v = 0.5 * (a[(long)i * lda + j] + a[(long)j * lda + i]);
  a[(long)i * lda + j] = v;
  a[(long)j * lda + i] = v;
}

__global__ void build_shifted_kernel(const double* __restrict__ t, const double* __restrict__ tm, int m, int ld,
                                     const double* __restrict__ sh, int pair, double* __restrict__ mats) {
  const int b = blockIdx.y;
  const int d = pair ? 2 * m : m;
  double* out = mats + (long)b * d * d;
  const double s = sh[b];
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < d * d; e += gridDim.x * blockDim.x) {
    const int i = e / d, j = e - i * d;
    double v;
    if (!pair) {
      v = t[(long)i * ld + j] - (i == j ? s : 0.0);
    } else {
      const int bi = i / m, bj = j / m, ii = i - bi * m, jj = j - bj * m;
      if (bi == 0 && bj == 0)
        v = t[(long)ii * ld + jj];
      else if (bi == 1 && bj == 1)
        v = tm[(long)ii * ld + jj];
      else
        v = (ii == jj) ? -s : 0.0;
    }
    out[e] = v;
  }
}

__global__ void copy_block_kernel(const double* __restrict__ src, int lds, int rows, int cols, double* __restrict__ dst,
                                  int ldd) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rows * cols) return;
  const int i = t / cols, j = t - i * cols;
  dst[(long)i * ldd + j] = src[(long)i * lds + j];
}

}  // namespace

void small_eigh(double* a, int m, int lda, double* w, double* q, double* work, hipStream_t s) {
  if (m <= 0) return;
  RID_CHECK(m <= MAXM, RID_ERR_SHAPE, "projected dimension above 1024");
  hipLaunchKernelGGL(jacobi_kernel, dim3(1), dim3(DB), 0, s, a, m, lda, w, q, work);
  RID_HIP(hipGetLastError());
}

size_t small_syevx_work(int m, int k) { return (size_t)3 * m + (size_t)6 * m * k + 2 * (size_t)m + 64; }

void small_syevx(double* a, int m, int lda, int k, double* w, double* q, int ldq, double* work, hipStream_t s) {
  if (m <= 0 || k <= 0) return;
  RID_CHECK(m <= MAXM, RID_ERR_SHAPE, "projected dimension above 1024");
  RID_CHECK(k <= m && k <= DB, RID_ERR_SHAPE, "k must be <= m and <= 1024");
  hipLaunchKernelGGL(syevx_kernel, dim3(1), dim3(DB), 0, s, a, m, lda, k, w, q, ldq, work);
  RID_HIP(hipGetLastError());
}

void small_chol(double* a, int m, int lda, int* info, hipStream_t s) {
  if (m <= 0) return;
  if (m <= CHOL_SMALL)
    hipLaunchKernelGGL(chol_small_kernel, dim3(1), dim3(64), 0, s, a, m, lda, info);
  else if (m <= CHOL_BLK_MAX)
    hipLaunchKernelGGL(chol_blocked_kernel, dim3(1), dim3(DB), 0, s, a, m, lda, info);
  else
    hipLaunchKernelGGL(chol_kernel, dim3(1), dim3(DB), 0, s, a, m, lda, info);
  RID_HIP(hipGetLastError());
}

void small_lu_solve(double* mats, double* rhs, int m, int nb, hipStream_t s) {
  if (m <= 0 || nb <= 0) return;
  hipLaunchKernelGGL(lu_solve_kernel, dim3(nb), dim3(DB), 0, s, mats, rhs, m);
  RID_HIP(hipGetLastError());
}

void small_lu_solve_cm(double* mats, double* rhs, int m, int nb, hipStream_t s) {
  if (m <= 0 || nb <= 0) return;
  if (m <= LU_LDS_MAX)
    hipLaunchKernelGGL(lu_lds_kernel, dim3(nb), dim3(LB), 0, s, mats, rhs, m);
  else if (m <= LU_BLK_MAX)
    hipLaunchKernelGGL(lu_blocked_kernel, dim3(nb), dim3(LB), 0, s, mats, rhs, m);
  else
    hipLaunchKernelGGL(lu_cm_kernel, dim3(nb), dim3(LB), 0, s, mats, rhs, m);
  RID_HIP(hipGetLastError());
}

void pair_systems_build(const double* P, const double* tp, const double* tm, int ld, int m, const int* sys_b,
                        const int* sys_type, const double* sys_shift, int nsys, const double* g, int ldg,
                        const double* tg, double* mats, double* rhs, hipStream_t s) {
  if (m <= 0 || nsys <= 0) return;
  RID_CHECK(nsys < 65536, RID_ERR_SHAPE, "too many pair systems");
  dim3 grid((unsigned)std::min(ceil_div(m * m, 256), 256), (unsigned)nsys);
  hipLaunchKernelGGL(pair_mats_kernel, grid, dim3(256), 0, s, P, tp, tm, ld, m, sys_type, sys_shift, mats);
  hipLaunchKernelGGL(pair_rhs_kernel, dim3(ceil_div(nsys * m, 256)), dim3(256), 0, s, g, ldg, tg, sys_b, sys_type,
                     sys_shift, nsys, m, rhs);
  RID_HIP(hipGetLastError());
}

void pair_systems_unpack(double* g, int ldg, const double* sol, const double* yt, const int* sys_b,
                         const int* sys_type, const double* sys_shift, int nsys, int m, hipStream_t s) {
  if (m <= 0 || nsys <= 0) return;
  hipLaunchKernelGGL(pair_unpack_kernel, dim3(ceil_div(nsys * m, 256)), dim3(256), 0, s, g, ldg, sol, yt, sys_b,
                     sys_type, sys_shift, nsys, m);
  RID_HIP(hipGetLastError());
}

void small_gemm(int ta, int tb, int m, int n, int k, double alpha, const double* A, int lda, const double* B, int ldb,
                double beta, double* C, int ldc, hipStream_t s) {
  if (m <= 0 || n <= 0) return;
  dim3 grid((unsigned)ceil_div(n, 16), (unsigned)ceil_div(m, 16));
  hipLaunchKernelGGL(small_gemm_kernel, grid, dim3(256), 0, s, ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc);
  RID_HIP(hipGetLastError());
}

void small_trinv_lower(const double* L, int m, int ldl, double* G, int ldg, hipStream_t s) {
  if (m <= 0) return;
  hipLaunchKernelGGL(trinv_lower_kernel, dim3(ceil_div(m, 64)), dim3(64), 0, s, L, m, ldl, G, ldg);
  RID_HIP(hipGetLastError());
}

void build_schur(const double* t, int ldt, const double* w, int ldw, int m, const double* sh, int nb, double* mats,
                 hipStream_t s) {
  if (m <= 0 || nb <= 0) return;
  dim3 grid((unsigned)std::min(ceil_div(m * m, 256), 1024), (unsigned)nb);
  hipLaunchKernelGGL(build_schur_kernel, grid, dim3(256), 0, s, t, ldt, w, ldw, m, sh, mats);
  RID_HIP(hipGetLastError());
}

void rows_axpy(const double* x, int ldx, const double* y, int ldy, const double* sh, int nb, int m, double* out,
               int ldo, hipStream_t s) {
  if (m <= 0 || nb <= 0) return;
  hipLaunchKernelGGL(rows_axpy_kernel, dim3(ceil_div(nb * m, 256)), dim3(256), 0, s, x, ldx, y, ldy, sh, nb, m, out,
                     ldo);
  RID_HIP(hipGetLastError());
}

void small_symmetrize(double* a, int m, int lda, hipStream_t s) {
  if (m <= 1) return;
  hipLaunchKernelGGL(symmetrize_kernel, dim3(ceil_div(m * m, 256)), dim3(256), 0, s, a, m, lda);
  RID_HIP(hipGetLastError());
}

void build_shifted(const double* t, const double* tm, int m, int ld, const double* sh, int nb, int pair, double* mats,
                   hipStream_t s) {
  if (m <= 0 || nb <= 0) return;
  const int d = pair ? 2 * m : m;
  dim3 grid((unsigned)std::min(ceil_div(d * d, 256), 1024), (unsigned)nb);
  hipLaunchKernelGGL(build_shifted_kernel, grid, dim3(256), 0, s, t, tm, m, ld, sh, pair, mats);
  RID_HIP(hipGetLastError());
}

void copy_block(const double* src, int lds, int rows, int cols, double* dst, int ldd, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return;
  hipLaunchKernelGGL(copy_block_kernel, dim3(ceil_div(rows * cols, 256)), dim3(256), 0, s, src, lds, rows, cols, dst,
                     ldd);
  RID_HIP(hipGetLastError());
}

}  // namespace rid

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
// parallel.  Sweeps stop when the squared off-diagonal Frobenius norm falls
// below 1e-30 of the squared full norm.
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
  __shared__ double red[16];
  __shared__ double cs[MAXM / 2], sn[MAXM / 2];
  __shared__ int pp[MAXM / 2], qq[MAXM / 2];
  __shared__ int rank[MAXM];
  __shared__ int stop;
  const int tid = threadIdx.x;
  for (int t = tid; t < m * m; t += DB) q[t] = (t / m == t % m) ? 1.0 : 0.0;
  const int mm = m + (m & 1);
  const int npair = mm / 2;
  __syncthreads();
  for (int sweep = 0; sweep < 60 && m > 1; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int t = tid; t < m * m; t += DB) {
      const int i = t / m, j = t % m;
      const double v = a[(long)i * lda + j];
      tot += v * v;
      if (i != j) off += v * v;
    }
    off = block_sum(off, red);
    tot = block_sum(tot, red);
    if (tid == 0) stop = (off <= 1e-30 * tot) || tot == 0.0;
    __syncthreads();
    if (stop) break;
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
          if (apq != 0.0) {
            const double app = a[(long)p * lda + p], aqq = a[(long)qv * lda + qv];
            const double tau = (aqq - app) / (2.0 * apq);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
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

// Cholesky, left-looking by columns.
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

void small_chol(double* a, int m, int lda, int* info, hipStream_t s) {
  if (m <= 0) return;
  hipLaunchKernelGGL(chol_kernel, dim3(1), dim3(DB), 0, s, a, m, lda, info);
  RID_HIP(hipGetLastError());
}

void small_lu_solve(double* mats, double* rhs, int m, int nb, hipStream_t s) {
  if (m <= 0 || nb <= 0) return;
  hipLaunchKernelGGL(lu_solve_kernel, dim3(nb), dim3(DB), 0, s, mats, rhs, m);
  RID_HIP(hipGetLastError());
}

void small_gemm(int ta, int tb, int m, int n, int k, double alpha, const double* A, int lda, const double* B, int ldb,
                double beta, double* C, int ldc, hipStream_t s) {
  if (m <= 0 || n <= 0) return;
  dim3 grid((unsigned)ceil_div(n, 16), (unsigned)ceil_div(m, 16));
  hipLaunchKernelGGL(small_gemm_kernel, grid, dim3(256), 0, s, ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc);
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

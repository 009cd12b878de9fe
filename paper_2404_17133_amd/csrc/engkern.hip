// Memory-bound FP64 kernels of the Krylov engine.
//
// gram: C = V W^T for a tall block V (m x N) and a few vectors W (n x N).
// Each workgroup takes an 8 x 8 tile of (i, j) and one chunk of the long
// index; every lane accumulates its 64 products in registers over a strided
// walk of the chunk, the wave then folds the 64 accumulators onto 64 lanes
// with a halving butterfly (63 shuffles instead of 64 reductions), and the 4
// waves add through LDS.  A second kernel sums the chunk partials.
// combo: Out = beta Out + alpha c^T V, one lane per long index, the
// coefficients read with wave-uniform (scalar) loads.
#include <algorithm>

#include "engkern.hpp"

namespace rid {
namespace {

constexpr int TI = 8, TJ = 8;

inline int grid1(long n, int block = 256) {
  long g = (n + block - 1) / block;
  return (int)std::max<long>(1, std::min<long>(g, 65536));
}

int gram_chunks(int m, int n, long N) {
  const long tiles = (long)ceil_div(m, TI) * ceil_div(n, TJ);
  long ch = (2048 + tiles - 1) / tiles;
  ch = std::min<long>(ch, std::max<long>(1, (N + 1023) / 1024));
  return (int)std::max<long>(1, std::min<long>(ch, 4096));
}

// One halving step of the butterfly: 2*O live accumulators become O.  The
// step width is a template constant so that every array index is known at
// compile time and the accumulators stay in registers.
template <int O>
__device__ inline void fold_step(double (&a)[64], int lane) {
  const bool upper = (lane & O) != 0;
#pragma unroll
  for (int q = 0; q < O; ++q) {
    const double send = upper ? a[q] : a[q + O];
    const double keep = upper ? a[q + O] : a[q];
    a[q] = keep + __shfl_xor(send, O, 64);
  }
}

__device__ inline void fold64(double (&a)[64], int lane) {
  fold_step<32>(a, lane);
  fold_step<16>(a, lane);
  fold_step<8>(a, lane);
  fold_step<4>(a, lane);
  fold_step<2>(a, lane);
  fold_step<1>(a, lane);
}

__global__ __launch_bounds__(256) void gram_part_kernel(const double* __restrict__ V, long ldv, int m,
                                                        const double* __restrict__ W, long ldw, int n, long N,
                                                        long chunk, double* __restrict__ part) {
  const int i0 = blockIdx.x * TI, j0 = blockIdx.y * TJ;
  const long k0 = blockIdx.z * chunk;
  const long k1 = min(N, k0 + chunk);
  double acc[64];
#pragma unroll
  for (int q = 0; q < 64; ++q) acc[q] = 0.0;
  const double* vr[TI];
  const double* wr[TJ];
#pragma unroll
  for (int a = 0; a < TI; ++a) vr[a] = V + (long)min(i0 + a, m - 1) * ldv;
#pragma unroll
  for (int b = 0; b < TJ; ++b) wr[b] = W + (long)min(j0 + b, n - 1) * ldw;
  for (long k = k0 + threadIdx.x; k < k1; k += 256) {
    double v[TI], w[TJ];
#pragma unroll
    for (int a = 0; a < TI; ++a) v[a] = vr[a][k];
#pragma unroll
    for (int b = 0; b < TJ; ++b) w[b] = wr[b][k];
#pragma unroll
    for (int a = 0; a < TI; ++a)
#pragma unroll
      for (int b = 0; b < TJ; ++b) acc[a * TJ + b] += v[a] * w[b];
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  fold64(acc, lane);
  __shared__ double red[4][64];
  red[wave][lane] = acc[0];
  __syncthreads();
  if (threadIdx.x < 64) {
    const double s = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
    const int i = i0 + threadIdx.x / TJ, j = j0 + threadIdx.x % TJ;
    if (i < m && j < n) part[((long)blockIdx.z * m + i) * n + j] = s;
  }
}

__global__ void sum_parts_kernel(const double* __restrict__ part, int nch, int m, int n, double* __restrict__ C,
                                 int ldc) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m * n) return;
  const int i = t / n, j = t % n;
  double s = 0.0;
  for (int c = 0; c < nch; ++c) s += part[((long)c * m + i) * n + j];
  C[(long)i * ldc + j] = s;
}

// The same reduction for few outputs: one wavefront per output, the lanes
// take the chunks in turn and a fixed butterfly adds their sums, so that a
// small Gram matrix does not wait on one thread's serial loop.
__global__ __launch_bounds__(256) void sum_parts_wave_kernel(const double* __restrict__ part, int nch, int m, int n,
                                                             double* __restrict__ C, int ldc) {
  const int lane = threadIdx.x & 63;
  const long t = blockIdx.x * 4L + (threadIdx.x >> 6);
  if (t >= (long)m * n) return;  // uniform per wavefront
  const int i = (int)(t / n), j = (int)(t % n);
  double s = 0.0;
  for (int c = lane; c < nch; c += 64) s += part[((long)c * m + i) * n + j];
  s = wave_sum(s);
  if (lane == 0) C[(long)i * ldc + j] = s;
}

__global__ __launch_bounds__(256) void norm_part_kernel(const double* __restrict__ W, long ldw, int n, long N,
                                                        long chunk, double* __restrict__ part) {
  const int j = blockIdx.y;
  const long k0 = blockIdx.x * chunk, k1 = min(N, k0 + chunk);
  const double* w = W + (long)j * ldw;
  double s = 0.0;
  for (long k = k0 + threadIdx.x; k < k1; k += 256) s += w[k] * w[k];
  s = wave_sum(s);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[(long)j * gridDim.x + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void norm_final_kernel(const double* __restrict__ part, int nch, int n, double* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double s = 0.0;
  for (int c = 0; c < nch; ++c) s += part[(long)j * nch + c];
  out[j] = sqrt(s);
}

template <int NJ>
__global__ __launch_bounds__(256) void combo_kernel(const double* __restrict__ V, long ldv, int m,
                                                    const double* __restrict__ c, int csi, int csj, int n, long N,
                                                    double alpha, double beta, double* __restrict__ Out, long ldo) {
  const long k = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const int j0 = blockIdx.y * NJ;
  if (k >= N) return;
  double acc[NJ];
#pragma unroll
  for (int q = 0; q < NJ; ++q) acc[q] = 0.0;
  for (int i = 0; i < m; ++i) {
    const double v = V[(long)i * ldv + k];
    const double* ci = c + (long)i * csi + (long)j0 * csj;
#pragma unroll
    for (int q = 0; q < NJ; ++q) acc[q] += (j0 + q < n ? ci[(long)q * csj] : 0.0) * v;
  }
#pragma unroll
  for (int q = 0; q < NJ; ++q) {
    if (j0 + q < n) {
      double* o = Out + (long)(j0 + q) * ldo + k;
      *o = (beta == 0.0 ? 0.0 : beta * *o) + alpha * acc[q];
    }
  }
}

__global__ void scale_cols_kernel(double* W, long ldw, int n, long N, const double* __restrict__ sc, int inv) {
  const long total = (long)n * N;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const int j = (int)(t / N);
    const long k = t - (long)j * N;
    double f = sc[j];
    if (inv) f = f != 0.0 ? 1.0 / f : 1.0;
    W[(long)j * ldw + k] *= f;
  }
}

__global__ void residual_kernel(const double* __restrict__ AX, const double* __restrict__ X, long ld, int n, long N,
                                const double* __restrict__ om, double* __restrict__ R) {
  const long total = (long)n * N;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const int j = (int)(t / N);
    const long k = t - (long)j * N;
    const long o = (long)j * ld + k;
    R[o] = AX[o] - om[j] * X[o];
  }
}

__global__ void residual_pair_kernel(const double* __restrict__ Pz, const double* __restrict__ Zp,
                                     const double* __restrict__ Mzp, const double* __restrict__ Z, long ld, int n,
                                     long N, const double* __restrict__ om, double* __restrict__ R1,
                                     double* __restrict__ R2) {
  const long total = (long)n * N;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const int j = (int)(t / N);
    const long k = t - (long)j * N;
    const long o = (long)j * ld + k;
    R1[o] = Pz[o] - om[j] * Zp[o];
    R2[o] = Mzp[o] - om[j] * Z[o];
  }
}

__device__ inline double guard(double d) {
  if (fabs(d) < 1e-8) return d < 0.0 ? -1e-8 : 1e-8;
  return d;
}

__global__ void diag_tda_kernel(const double* __restrict__ de, const double* __restrict__ r, long ldr, int n, long N,
                                const double* __restrict__ sh, const int* __restrict__ idx, double* __restrict__ out,
                                long ldo) {
  const long total = (long)n * N;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const int j = (int)(t / N);
    const long k = t - (long)j * N;
    const int src = idx ? idx[j] : j;
    out[(long)j * ldo + k] = r[(long)src * ldr + k] / guard(de[k] - sh[src]);
  }
}

__global__ void diag_pair_kernel(const double* __restrict__ de, const double* __restrict__ r1,
                                 const double* __restrict__ r2, long ldr, int n, long N, const double* __restrict__ sh,
                                 const int* __restrict__ idx, double* __restrict__ d1, double* __restrict__ d2,
                                 long ldo) {
  const long total = (long)n * N;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const int j = (int)(t / N);
    const long k = t - (long)j * N;
    const int src = idx ? idx[j] : j;
    const double s = sh[src];
    const double den = guard(de[k] - s) * (de[k] + s);
    const double a = r1[(long)src * ldr + k], b = r2[(long)src * ldr + k];
    d1[(long)j * ldo + k] = (de[k] * a + s * b) / den;
    d2[(long)j * ldo + k] = (s * a + de[k] * b) / den;
  }
}

__global__ void axpby_kernel(const double* __restrict__ x, const double* __restrict__ y, long ld, int n, long N,
                             const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ out,
                             long ldo) {
  const long total = (long)n * N;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const int j = (int)(t / N);
    const long k = t - (long)j * N;
    double v = 0.0;
    if (a) v += a[j] * x[(long)j * ld + k];
    if (b) v += b[j] * y[(long)j * ld + k];
    out[(long)j * ldo + k] = v;
  }
}

__global__ void gather_kernel(const double* __restrict__ src, long lds, const int* __restrict__ idx, int n, long N,
                              double* __restrict__ dst, long ldd) {
  const long total = (long)n * N;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const int j = (int)(t / N);
    const long k = t - (long)j * N;
    const int s = idx ? idx[j] : j;
    dst[(long)j * ldd + k] = src[(long)s * lds + k];
  }
}

__global__ void unit_kernel(const int* __restrict__ pos, int n, long N, double* __restrict__ out, long ldo) {
  const long total = (long)n * N;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const int j = (int)(t / N);
    const long k = t - (long)j * N;
    out[(long)j * ldo + k] = (k == pos[j]) ? 1.0 : 0.0;
  }
}

__global__ void resid3_kernel(const double* __restrict__ a, const double* __restrict__ b,
                              const double* __restrict__ c, long ld, int n, long N, const double* __restrict__ sh,
                              double* __restrict__ out, long ldo) {
  const long total = (long)n * N;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const int j = (int)(t / N);
    const long k = t - (long)j * N;
    const long o = (long)j * ld + k;
    double v = a[o] - sh[j] * b[o];
    if (c) v -= c[o];
    out[(long)j * ldo + k] = v;
  }
}

__global__ void proj_update_kernel(double* a, int lda, int m, int m0, const double* __restrict__ c1,
                                   const double* __restrict__ c2) {
  const int nn = m - m0;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m * nn) return;
  const int i = t / nn, jj = t - i * nn, j = m0 + jj;
  const double v = 0.5 * (c1[t] + c2[t]);
  a[(long)i * lda + j] = v;
  a[(long)j * lda + i] = v;
}

__global__ void scale_copy_kernel(const double* __restrict__ src, long n, double alpha, double* __restrict__ dst) {
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x)
    dst[t] = alpha * src[t];
}

// dst = src / r when r = *rp >= tol, else dst = 0 (a dropped direction).
__global__ void accept_scale_kernel(const double* __restrict__ src, long n, const double* __restrict__ rp, double tol,
                                    double* __restrict__ dst) {
  const double r = *rp;
  const bool ok = r >= tol;
  const double alpha = ok ? 1.0 / r : 0.0;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x)
    dst[t] = ok ? alpha * src[t] : 0.0;
}

__global__ void chol_check_pack_kernel(const double* __restrict__ l, int n, int ldl, const double* __restrict__ nrm,
                                       const int* __restrict__ info, double* __restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) {
    out[t] = l[(long)t * ldl + t];
    out[n + t] = nrm[t];
  }
  if (t == 0) out[2 * n] = (double)info[0];
}

}  // namespace

void chol_check_pack(const double* l, int n, int ldl, const double* nrm, const int* info, double* out, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(chol_check_pack_kernel, dim3((n + 255) / 256), dim3(256), 0, s, l, n, ldl, nrm, info, out);
  RID_HIP(hipGetLastError());
}

void accept_scale(const double* src, long n, const double* r, double tol, double* dst, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(accept_scale_kernel, dim3(grid1(n)), dim3(256), 0, s, src, n, r, tol, dst);
  RID_HIP(hipGetLastError());
}

size_t gram_part_elems(int m, int n, long N) { return (size_t)gram_chunks(m, n, N) * std::max(m, 1) * std::max(n, 1); }

void gram(const double* V, long ldv, int m, const double* W, long ldw, int n, long N, double* C, int ldc,
          const RedScratch& rs, hipStream_t s) {
  if (m <= 0 || n <= 0) return;
  const int nch = gram_chunks(m, n, N);
  RID_CHECK((size_t)nch * m * n <= rs.part_elems, RID_ERR_INTERNAL, "gram: scratch too small");
  const long chunk = (N + nch - 1) / nch;
  dim3 grid((unsigned)ceil_div(m, TI), (unsigned)ceil_div(n, TJ), (unsigned)nch);
  RID_CHECK(ceil_div(m, TI) < 65536 && ceil_div(n, TJ) < 65536, RID_ERR_SHAPE, "gram: too many vectors");
  hipLaunchKernelGGL(gram_part_kernel, grid, dim3(256), 0, s, V, ldv, m, W, ldw, n, N, chunk, rs.part);
  if ((long)m * n < 1024)
    hipLaunchKernelGGL(sum_parts_wave_kernel, dim3(ceil_div(m * n, 4)), dim3(256), 0, s, rs.part, nch, m, n, C, ldc);
  else
    hipLaunchKernelGGL(sum_parts_kernel, dim3(ceil_div(m * n, 256)), dim3(256), 0, s, rs.part, nch, m, n, C, ldc);
  RID_HIP(hipGetLastError());
}

void combo(const double* V, long ldv, int m, const double* c, int csi, int csj, int n, long N, double alpha,
           double beta, double* Out, long ldo, hipStream_t s) {
  if (n <= 0 || N <= 0) return;
  if (m <= 0 && beta == 1.0) return;
  constexpr int NJ = 8;
  dim3 grid((unsigned)((N + 255) / 256), (unsigned)ceil_div(n, NJ));
  hipLaunchKernelGGL((combo_kernel<NJ>), grid, dim3(256), 0, s, V, ldv, std::max(m, 0), c, csi, csj, n, N, alpha,
                     beta, Out, ldo);
  RID_HIP(hipGetLastError());
}

void resid3(const double* a, const double* b, const double* c, long ld, int n, long N, const double* sh,
            double* out, long ldo, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(resid3_kernel, dim3(grid1((long)n * N)), dim3(256), 0, s, a, b, c, ld, n, N, sh, out, ldo);
  RID_HIP(hipGetLastError());
}

void proj_update(double* a, int lda, int m, int m0, const double* c1, const double* c2, hipStream_t s) {
  const int nn = m - m0;
  if (nn <= 0) return;
  hipLaunchKernelGGL(proj_update_kernel, dim3(ceil_div(m * nn, 256)), dim3(256), 0, s, a, lda, m, m0, c1, c2);
  RID_HIP(hipGetLastError());
}

void col_norms(const double* W, long ldw, int n, long N, double* out, const RedScratch& rs, hipStream_t s) {
  if (n <= 0) return;
  int nch = (int)std::max<long>(1, std::min<long>(256, (N + 4095) / 4096));
  RID_CHECK((size_t)nch * n <= rs.part_elems, RID_ERR_INTERNAL, "col_norms: scratch too small");
  const long chunk = (N + nch - 1) / nch;
  hipLaunchKernelGGL(norm_part_kernel, dim3(nch, n), dim3(256), 0, s, W, ldw, n, N, chunk, rs.part);
  hipLaunchKernelGGL(norm_final_kernel, dim3(ceil_div(n, 64)), dim3(64), 0, s, rs.part, nch, n, out);
  RID_HIP(hipGetLastError());
}

void scale_cols(double* W, long ldw, int n, long N, const double* sc, int inv, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(scale_cols_kernel, dim3(grid1((long)n * N)), dim3(256), 0, s, W, ldw, n, N, sc, inv);
  RID_HIP(hipGetLastError());
}

void residual(const double* AX, const double* X, long ld, int n, long N, const double* om, double* R, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(residual_kernel, dim3(grid1((long)n * N)), dim3(256), 0, s, AX, X, ld, n, N, om, R);
  RID_HIP(hipGetLastError());
}

void residual_pair(const double* Pz, const double* Zp, const double* Mzp, const double* Z, long ld, int n, long N,
                   const double* om, double* R1, double* R2, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(residual_pair_kernel, dim3(grid1((long)n * N)), dim3(256), 0, s, Pz, Zp, Mzp, Z, ld, n, N, om,
                     R1, R2);
  RID_HIP(hipGetLastError());
}

void diag_tda(const double* de, const double* r, long ldr, int n, long N, const double* sh, const int* idx,
              double* out, long ldo, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(diag_tda_kernel, dim3(grid1((long)n * N)), dim3(256), 0, s, de, r, ldr, n, N, sh, idx, out,
                     ldo);
  RID_HIP(hipGetLastError());
}

void diag_pair(const double* de, const double* r1, const double* r2, long ldr, int n, long N, const double* sh,
               const int* idx, double* d1, double* d2, long ldo, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(diag_pair_kernel, dim3(grid1((long)n * N)), dim3(256), 0, s, de, r1, r2, ldr, n, N, sh, idx, d1,
                     d2, ldo);
  RID_HIP(hipGetLastError());
}

void axpby_cols(const double* x, const double* y, long ld, int n, long N, const double* a, const double* b,
                double* out, long ldo, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(axpby_kernel, dim3(grid1((long)n * N)), dim3(256), 0, s, x, y, ld, n, N, a, b, out, ldo);
  RID_HIP(hipGetLastError());
}

void gather_cols(const double* src, long lds, const int* idx, int n, long N, double* dst, long ldd, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(gather_kernel, dim3(grid1((long)n * N)), dim3(256), 0, s, src, lds, idx, n, N, dst, ldd);
  RID_HIP(hipGetLastError());
}

void unit_vectors(const int* pos, int n, long N, double* out, long ldo, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(unit_kernel, dim3(grid1((long)n * N)), dim3(256), 0, s, pos, n, N, out, ldo);
  RID_HIP(hipGetLastError());
}

void scale_copy(const double* src, long n, double alpha, double* dst, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(scale_copy_kernel, dim3(grid1(n)), dim3(256), 0, s, src, n, alpha, dst);
  RID_HIP(hipGetLastError());
}

}  // namespace rid

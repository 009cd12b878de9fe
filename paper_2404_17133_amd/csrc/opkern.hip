// Memory-bound kernels around the operator contractions: vector layout
// preparation, Coulomb back-projection, reduction of split partial sums and
// the final combination into A x, (A+B) x, (A-B) x (or the ris analogues).
#include "opkern.hpp"

namespace rid {
namespace {

template <typename E>
__device__ inline E to_elem(double v);
template <>
__device__ inline double to_elem<double>(double v) { return v; }
template <>
__device__ inline float to_elem<float>(double v) { return (float)v; }
template <>
__device__ inline uint16_t to_elem<uint16_t>(double v) { return f32_to_bf16_bits((float)v); }

template <typename E>
__device__ inline double from_elem(E v);
template <>
__device__ inline double from_elem<double>(double v) { return v; }
template <>
__device__ inline double from_elem<float>(float v) { return (double)v; }
template <>
__device__ inline double from_elem<uint16_t>(uint16_t v) { return (double)bf16_bits_to_f32(v); }

// x (nvec x N, f64) -> xc (nvec x N), xa (nvec x no_a x kv), xt (nvec x kv x no_a): the
// window [i0, i0 + no_a) x [0, nv_a) of every vector, with the virtual index
// padded to kv >= nv_a (nv_a <= kv <= nv) by zeros, so that the exchange
// contractions over it can use 16-byte loads.
template <typename E>
__global__ void prep_x_kernel(const double* __restrict__ x, int nvec, int no, int nv, int i0, int no_a,
                              int nv_a, int kv, E* __restrict__ xc, E* __restrict__ xa, E* __restrict__ xt) {
  const long n = (long)no * nv;
  const long total = (long)nvec * n;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const int v = (int)(t / n);
    const long ia = t - (long)v * n;
    const int i = (int)(ia / nv);
    const int a = (int)(ia - (long)i * nv);
    const E e = to_elem<E>(x[t]);
    if (xc) xc[t] = e;
    const int j = i - i0;
    if (j >= 0 && j < no_a && a < kv) {
      const E ew = a < nv_a ? e : to_elem<E>(0.0);
      if (xa) xa[((long)v * no_a + j) * kv + a] = ew;
      if (xt) xt[((long)v * kv + a) * no_a + j] = ew;
    }
  }
}

// out[i] = sum_s part[s * stride + i], accumulated in f64
template <typename A>
__global__ void reduce_splits_kernel(const A* __restrict__ part, int ns, long stride, long n,
                                     double* __restrict__ out) {
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int q = 0; q < ns; ++q) s += (double)part[q * stride + t];
    out[t] = s;
  }
}

// J[v][ia] = sum_P t[v][P] * b[P][ia]; NVB vectors per blockIdx.y, rows
// [z * pch, (z + 1) * pch) of P per blockIdx.z, f64 accumulation.  t is read
// with wave-uniform addresses (scalar loads); b is read once per vector
// group, coalesced along ia.  With several P ranges each writes its partial
// sums at out + z * nvec * n (summed afterwards); with one, out is J.
template <typename E, int NVB>
__global__ __launch_bounds__(256) void coul_bwd_kernel(const double* __restrict__ t, const E* __restrict__ b,
                                                       int naux, long n, int nvec, int pch, double* __restrict__ out) {
  const long ia = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const int v0 = blockIdx.y * NVB;
  const int p0 = blockIdx.z * pch, p1 = min(naux, p0 + pch);
  double* o = out + (long)blockIdx.z * nvec * n;
  double acc[NVB];
#pragma unroll
  for (int q = 0; q < NVB; ++q) acc[q] = 0.0;
  if (ia < n) {
    // several rows of b in flight per thread: the loop is latency-bound
#pragma unroll 8
    for (int p = p0; p < p1; ++p) {
      const double bv = from_elem<E>(b[(long)p * n + ia]);
#pragma unroll
      for (int q = 0; q < NVB; ++q) {
        const int v = v0 + q < nvec ? v0 + q : nvec - 1;
        acc[q] += t[(long)v * naux + p] * bv;
      }
    }
#pragma unroll
    for (int q = 0; q < NVB; ++q)
      if (v0 + q < nvec) o[(long)(v0 + q) * n + ia] = acc[q];
  }
}

// Sum of the split partials of an exchange product at (v, i, a).  The
// partial layout is [s][(i - i0) * nvec + v][a] with row length nv_a.
template <typename A>
__device__ inline double exch_sum(const A* __restrict__ wp, int ns, long sstride, int nvec, int nv_a, int v, int ii,
                                  int a) {
  const long off = ((long)ii * nvec + v) * nv_a + a;
  double s = 0.0;
  for (int q = 0; q < ns; ++q) s += (double)wp[q * sstride + off];
  return s;
}

template <typename A>
__global__ void combine_kernel(CombineArgs c, const A* __restrict__ wp, const A* __restrict__ wpp) {
  const long n = (long)c.no * c.nv;
  const long total = (long)c.nvec * n;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const int v = (int)(t / n);
    const long ia = t - (long)v * n;
    const int i = (int)(ia / c.nv);
    const int a = (int)(ia - (long)i * c.nv);
    const double dx = c.de[ia] * c.x[t];
    const double jj = c.j ? c.j[t] : 0.0;
    double w = 0.0, w2 = 0.0;
    const int ii = i - c.i0;
    if (ii >= 0 && ii < c.no_a && a < c.nv_a) {
      if (wp) w = exch_sum(wp, c.ns_w, c.sstride, c.nvec, c.nv_a, v, ii, a);
      if (wpp) w2 = exch_sum(wpp, c.ns_wp, c.sstride, c.nvec, c.nv_a, v, ii, a);
    }
    if (c.pair) {
      c.y[t] = dx + c.cj * jj - c.a_x * (w + w2);
      c.y2[t] = dx - c.a_x * (w - w2);
    } else {
      c.y[t] = dx + c.cj * jj - c.a_x * w;
    }
  }
}

template <typename S, typename E>
__global__ void cast_kernel(const S* __restrict__ src, long n, E* __restrict__ dst) {
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x)
    dst[t] = to_elem<E>(src[t]);
}

// dst[p][c][r] = src[p][r][c] for an (rows x cols) slice per p, 32x32 LDS tiles.
template <typename S, typename E>
__global__ void transpose_kernel(const S* __restrict__ src, int rows, int cols, E* __restrict__ dst) {
  __shared__ S tile[32][33];
  const long p = blockIdx.z;
  const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
  const S* s = src + p * (long)rows * cols;
  E* d = dst + p * (long)rows * cols;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 256 threads: 32 x 8
  for (int k = ty; k < 32; k += 8) {
    const int r = r0 + k, c = c0 + tx;
    tile[k][tx] = (r < rows && c < cols) ? s[(long)r * cols + c] : S(0);
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int c = c0 + k, r = r0 + tx;
    if (r < rows && c < cols) d[(long)c * rows + r] = to_elem<E>(tile[tx][k]);
  }
}

inline int grid_for(long n, int block = 256) {
  long g = (n + block - 1) / block;
  return (int)(g > 65536 ? 65536 : (g < 1 ? 1 : g));
}

}  // namespace

template <typename E>
void prep_x(const double* x, int nvec, int no, int nv, int i0, int no_a, int nv_a, int kv, E* xc, E* xa, E* xt,
            hipStream_t s) {
  const long total = (long)nvec * no * nv;
  if (total == 0) return;
  RID_CHECK(kv >= nv_a && kv <= nv, RID_ERR_INTERNAL, "prep_x: padded window out of range");
  hipLaunchKernelGGL(prep_x_kernel<E>, dim3(grid_for(total)), dim3(256), 0, s, x, nvec, no, nv, i0, no_a, nv_a, kv,
                     xc, xa, xt);
  RID_HIP(hipGetLastError());
}

template <typename A>
void reduce_splits(const A* part, int ns, long stride, long n, double* out, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(reduce_splits_kernel<A>, dim3(grid_for(n)), dim3(256), 0, s, part, ns, stride, n, out);
  RID_HIP(hipGetLastError());
}

int coul_bwd_splits(long n, int nvec, int naux) {
  // enough workgroups to keep every CU busy with several (b is streamed
  // once per vector group, so the ranges of P add only partial traffic)
  const long gx = (n + 255) / 256;
  const long gy = nvec <= 16 ? 1 : ceil_div(nvec, 24);
  long ns = (2048 + gx * gy - 1) / (gx * gy);
  ns = std::min<long>(ns, std::max(1, naux / 64));
  return (int)std::max<long>(1, std::min<long>(ns, 16));
}

template <typename E>
void coul_bwd(const double* t, const E* b, int naux, long n, int nvec, double* j, double* part, size_t part_elems,
              hipStream_t s) {
  if (n == 0 || nvec == 0) return;
  int ns = coul_bwd_splits(n, nvec, naux);
  if (!part || (size_t)ns * nvec * n > part_elems) ns = 1;
  const int pch = ceil_div(naux, ns);
  ns = ceil_div(naux, pch);
  double* out = ns > 1 ? part : j;
  // one pass over b per group of vectors: as few passes as the register
  // budget allows (b is the bulk of the traffic)
  const unsigned gx = (unsigned)((n + 255) / 256);
  if (nvec <= 8)
    hipLaunchKernelGGL((coul_bwd_kernel<E, 8>), dim3(gx, 1, ns), dim3(256), 0, s, t, b, naux, n, nvec, pch, out);
  else if (nvec <= 16)
    hipLaunchKernelGGL((coul_bwd_kernel<E, 16>), dim3(gx, 1, ns), dim3(256), 0, s, t, b, naux, n, nvec, pch, out);
  else
    hipLaunchKernelGGL((coul_bwd_kernel<E, 24>), dim3(gx, (unsigned)ceil_div(nvec, 24), ns), dim3(256), 0, s, t, b,
                       naux, n, nvec, pch, out);
  RID_HIP(hipGetLastError());
  if (ns > 1) reduce_splits<double>(part, ns, (long)nvec * n, (long)nvec * n, j, s);
}

template <typename A>
void combine(const CombineArgs& c, const A* wp, const A* wpp, hipStream_t s) {
  const long total = (long)c.nvec * c.no * c.nv;
  if (total == 0) return;
  hipLaunchKernelGGL(combine_kernel<A>, dim3(grid_for(total)), dim3(256), 0, s, c, wp, wpp);
  RID_HIP(hipGetLastError());
}

template <typename S, typename E>
void cast_copy(const S* src, long n, E* dst, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL((cast_kernel<S, E>), dim3(grid_for(n)), dim3(256), 0, s, src, n, dst);
  RID_HIP(hipGetLastError());
}

template <typename S, typename E>
void transpose_slices(const S* src, int np, int rows, int cols, E* dst, hipStream_t s) {
  if (np == 0 || rows == 0 || cols == 0) return;
  dim3 grid((unsigned)ceil_div(cols, 32), (unsigned)ceil_div(rows, 32), (unsigned)np);
  RID_CHECK(np < 65536 && ceil_div(rows, 32) < 65536, RID_ERR_SHAPE, "transpose: grid too large");
  hipLaunchKernelGGL((transpose_kernel<S, E>), grid, dim3(256), 0, s, src, rows, cols, dst);
  RID_HIP(hipGetLastError());
}

#define RID_INST_E(E)                                                                                   \
  template void prep_x<E>(const double*, int, int, int, int, int, int, int, E*, E*, E*, hipStream_t);  \
  template void coul_bwd<E>(const double*, const E*, int, long, int, double*, double*, size_t, hipStream_t); \
  template void cast_copy<double, E>(const double*, long, E*, hipStream_t);                             \
  template void cast_copy<float, E>(const float*, long, E*, hipStream_t);                               \
  template void transpose_slices<double, E>(const double*, int, int, int, E*, hipStream_t);             \
  template void transpose_slices<float, E>(const float*, int, int, int, E*, hipStream_t);
RID_INST_E(double)
RID_INST_E(float)
RID_INST_E(uint16_t)
#undef RID_INST_E
template void reduce_splits<double>(const double*, int, long, long, double*, hipStream_t);
template void reduce_splits<float>(const float*, int, long, long, double*, hipStream_t);
template void combine<double>(const CombineArgs&, const double*, const double*, hipStream_t);
template void combine<float>(const CombineArgs&, const float*, const float*, hipStream_t);

}  // namespace rid

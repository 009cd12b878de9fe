// Auxiliary-basis RI tensors from a molecule: the minimal auxiliary basis of
// the ris model (Sec. 2.2.2, Eq. TDDFT-ris_approx: one Gaussian shell per
// angular momentum l <= l_max on each atom, exponent theta / R_A^2) or any
// explicit list of s, p, d shells (a full fitting basis for the operator A).
//
//   K^P_pq = (pq|P) = sum_{mu nu} C_mu,p C_nu,q (mu nu|P),
//   (P|Q) = L L^T (Cholesky),   B = sqrt(kappa) L^-1 K,
// so that B^T B = K^T (P|Q)^-1 K (Eq. pqrs_approx with the metric folded in).
// Auxiliary functions are ordered s first, then p, then d (shells in their
// given order; p as x, y, z; d as the real solid harmonics xy, xz, yz,
// x^2 - y^2, 2 z^2 - x^2 - y^2): since L is lower triangular the leading
// rows of B are then the tensor of the s functions alone, the exchange part
// of the (d, s) design of Sec. 3.2.  Atomic orbitals are normalised s
// Gaussians; auxiliary functions are not normalised (B depends only on the
// space they span and their order).
//
// Integrals.  A Cartesian Gaussian is a derivative of an s Gaussian with
// respect to its centre: (x - C_x) g = q d g/dC_x, (x - C_x)(y - C_y) g =
// q^2 d^2 g/dC_x dC_y and (x - C_x)^2 g = q^2 d^2 g/dC_x^2 + q g with
// q = 1 / (2c) (the q g terms cancel in every real d function above).  The
// Coulomb integral of two s Gaussians (exponents a, c at A, C) is
//   2 pi^(5/2) / (a c sqrt(a + c)) F_0(omega |X|^2),  X = A - C,
//   omega = a c / (a + c),
// so every integral here is a sum of derivatives of G_0(X) = F_0(omega |X|^2)
// up to fourth order, each written in closed form through
// G_m = (-2 omega)^m F_m(omega |X|^2) (d G_m / d X_j = X_j G_{m+1}):
//   d_i G_0 = X_i G_1,   d_ij G_0 = delta_ij G_1 + X_i X_j G_2,   ...
// The product of two s orbitals is one s Gaussian (Gaussian product
// theorem), so a three-centre integral is a two-centre one.
//
// Boys function: F_4 by its positive series exp(-T) sum_k (2T)^k /
// ((9)(11)...(9 + 2k)) and downward recursion F_n = (2 T F_{n+1} +
// exp(-T)) / (2n + 1) for T < 30; above, F_0 = sqrt(pi / T) / 2 (erf = 1 to
// rounding) and upward recursion F_{n+1} = ((2n + 1) F_n - exp(-T)) / (2T).
#include <cmath>
#include <vector>

#include "auxint.hpp"
#include "engkern.hpp"
#include "gemm.hpp"
#include "opkern.hpp"

namespace rid {
namespace {

// One auxiliary function: centre, exponent, kind (0 s; 1..3 p x, y, z;
// 4..8 d xy, xz, yz, x^2-y^2, 2z^2-x^2-y^2).
struct AuxFn {
  double x, y, z, e;
  int kind;
  int pad;
};

__device__ inline void boys5(double t, double f[5]) {
  if (t < 30.0) {
    const double et = exp(-t);
    double term = 1.0 / 9.0, sum = term;
    for (int k = 1; k < 200; ++k) {
      term *= 2.0 * t / (9.0 + 2.0 * k);
      sum += term;
      if (term < 1e-17 * sum) break;
    }
    f[4] = et * sum;
    f[3] = (2.0 * t * f[4] + et) / 7.0;
    f[2] = (2.0 * t * f[3] + et) / 5.0;
    f[1] = (2.0 * t * f[2] + et) / 3.0;
    f[0] = 2.0 * t * f[1] + et;
  } else {
    const double et = exp(-t);
    f[0] = 0.5 * sqrt(M_PI / t);
    f[1] = (f[0] - et) / (2.0 * t);
    f[2] = (3.0 * f[1] - et) / (2.0 * t);
    f[3] = (5.0 * f[2] - et) / (2.0 * t);
    f[4] = (7.0 * f[3] - et) / (2.0 * t);
  }
}

__device__ inline double comp(const double x[3], int i) { return i == 0 ? x[0] : (i == 1 ? x[1] : x[2]); }
__device__ inline double dl(int i, int j) { return i == j ? 1.0 : 0.0; }

// d^n G_0 / dX_{i0} ... dX_{i(n-1)} for n <= 4 (indices 0..2), G[m] = G_m.
__device__ double dg(int n, int i, int j, int k, int l, const double x[3], const double g[5]) {
  if (n == 0) return g[0];
  if (n == 1) return comp(x, i) * g[1];
  const double xi = comp(x, i), xj = comp(x, j);
  if (n == 2) return dl(i, j) * g[1] + xi * xj * g[2];
  const double xk = comp(x, k);
  if (n == 3) return (dl(i, j) * xk + dl(i, k) * xj + dl(j, k) * xi) * g[2] + xi * xj * xk * g[3];
  const double xl = comp(x, l);
  return (dl(i, j) * dl(k, l) + dl(i, k) * dl(j, l) + dl(i, l) * dl(j, k)) * g[2] +
         (dl(i, j) * xk * xl + dl(i, k) * xj * xl + dl(i, l) * xj * xk + dl(j, k) * xi * xl + dl(j, l) * xi * xk +
          dl(k, l) * xi * xj) * g[3] +
         xi * xj * xk * xl * g[4];
}

// A function as a sum of up to three centre-derivative terms: coefficient
// (in powers of q = 1/(2e)) and up to two derivative directions.
struct Terms {
  int n;           // number of terms
  int ord[3];      // derivatives per term (0, 1 or 2)
  int d0[3], d1[3];
  double c[3];
};

__device__ Terms terms_of(int kind, double e) {
  const double q = 0.5 / e;
  Terms t{};
  switch (kind) {
    case 0: t.n = 1; t.ord[0] = 0; t.c[0] = 1.0; break;
    case 1: case 2: case 3: t.n = 1; t.ord[0] = 1; t.d0[0] = kind - 1; t.c[0] = q; break;
    case 4: t.n = 1; t.ord[0] = 2; t.d0[0] = 0; t.d1[0] = 1; t.c[0] = q * q; break;
    case 5: t.n = 1; t.ord[0] = 2; t.d0[0] = 0; t.d1[0] = 2; t.c[0] = q * q; break;
    case 6: t.n = 1; t.ord[0] = 2; t.d0[0] = 1; t.d1[0] = 2; t.c[0] = q * q; break;
    case 7:
      t.n = 2;
      t.ord[0] = 2; t.d0[0] = 0; t.d1[0] = 0; t.c[0] = q * q;
      t.ord[1] = 2; t.d0[1] = 1; t.d1[1] = 1; t.c[1] = -q * q;
      break;
    default:
      t.n = 3;
      t.ord[0] = 2; t.d0[0] = 2; t.d1[0] = 2; t.c[0] = 2.0 * q * q;
      t.ord[1] = 2; t.d0[1] = 0; t.d1[1] = 0; t.c[1] = -q * q;
      t.ord[2] = 2; t.d0[2] = 1; t.d1[2] = 1; t.c[2] = -q * q;
      break;
  }
  return t;
}

// Coulomb integral of function (kind_a, exponent a at A) and (kind_c,
// exponent c at C).  Derivatives act on A for the first function and on C
// for the second (d/dC = -d/dX).
__device__ double coulomb(int kind_a, double a, const double A[3], int kind_c, double c, const double C[3]) {
  const double x[3] = {A[0] - C[0], A[1] - C[1], A[2] - C[2]};
  const double om = a * c / (a + c);
  double f[5];
  boys5(om * (x[0] * x[0] + x[1] * x[1] + x[2] * x[2]), f);
  double g[5];
  double s = 1.0;
  for (int m = 0; m < 5; ++m) {
    g[m] = s * f[m];
    s *= -2.0 * om;
  }
  const Terms ta = terms_of(kind_a, a), tc = terms_of(kind_c, c);
  double acc = 0.0;
  for (int p = 0; p < ta.n; ++p)
    for (int r = 0; r < tc.n; ++r) {
      // gather the derivative directions of both terms (first's, then second's)
      const int na = ta.ord[p], nc = tc.ord[r];
      int idx0 = 0, idx1 = 0, idx2 = 0, idx3 = 0;
      int n = 0;
      if (na > 0) { idx0 = ta.d0[p]; n = 1; }
      if (na > 1) { idx1 = ta.d1[p]; n = 2; }
      const int c0 = tc.d0[r], c1 = tc.d1[r];
      if (nc > 0) {
        if (n == 0) idx0 = c0; else if (n == 1) idx1 = c0; else idx2 = c0;
        ++n;
      }
      if (nc > 1) {
        if (n == 1) idx1 = c1; else if (n == 2) idx2 = c1; else idx3 = c1;
        ++n;
      }
      const double sign = (nc & 1) ? -1.0 : 1.0;
      acc += ta.c[p] * tc.c[r] * sign * dg(n, idx0, idx1, idx2, idx3, x, g);
    }
  return 2.0 * pow(M_PI, 2.5) / (a * c * sqrt(a + c)) * acc;
}

__global__ void metric_kernel(const AuxFn* __restrict__ fn, int n, double* __restrict__ J) {
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < (long)n * n; t += (long)gridDim.x * blockDim.x) {
    const int p = (int)(t / n), q = (int)(t - (long)p * n);
    const AuxFn a = fn[p], c = fn[q];
    const double A[3] = {a.x, a.y, a.z}, C[3] = {c.x, c.y, c.z};
    J[t] = coulomb(a.kind, a.e, A, c.kind, c.e, C);
  }
}

// X[P][mu][nu] = (mu nu|P); ao: centre (x, y, z), exponent and norm per AO
__global__ void three_center_kernel(const double* __restrict__ ao, int nao, const AuxFn* __restrict__ fn, int naux,
                                    double* __restrict__ X) {
  const long per = (long)nao * nao;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < per * naux; t += (long)gridDim.x * blockDim.x) {
    const int P = (int)(t / per);
    const long mn = t - (long)P * per;
    const int mu = (int)(mn / nao), nu = (int)(mn - (long)mu * nao);
    const double* am = ao + 5L * mu;
    const double* an = ao + 5L * nu;
    const double a = am[3], b = an[3], p = a + b;
    const double d2 =
        (am[0] - an[0]) * (am[0] - an[0]) + (am[1] - an[1]) * (am[1] - an[1]) + (am[2] - an[2]) * (am[2] - an[2]);
    const double pref = am[4] * an[4] * exp(-a * b / p * d2);
    const double Pc[3] = {(a * am[0] + b * an[0]) / p, (a * am[1] + b * an[1]) / p, (a * am[2] + b * an[2]) / p};
    const AuxFn c = fn[P];
    const double C[3] = {c.x, c.y, c.z};
    X[t] = pref * coulomb(0, p, Pc, c.kind, c.e, C);
  }
}

// out blocks of B[P][(p, q)] (nmo x nmo per P): ia (no x nv), ij, ab
__global__ void split_blocks_kernel(const double* __restrict__ b, int naux, int no, int nv, double* __restrict__ bia,
                                    double* __restrict__ bij, double* __restrict__ bab) {
  const int nmo = no + nv;
  const long per = (long)nmo * nmo;
  const long total = per * naux;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const long P = t / per;
    const long pq = t - P * per;
    const int p = (int)(pq / nmo), q = (int)(pq - (long)p * nmo);
    const double v = b[t];
    if (p < no && q < no) bij[(P * no + p) * no + q] = v;
    else if (p < no) bia[(P * no + p) * nv + (q - no)] = v;
    else if (q >= no) bab[(P * nv + (p - no)) * nv + (q - no)] = v;
  }
}

inline unsigned grid_of(long n) { return (unsigned)std::max<long>(1, std::min<long>((n + 255) / 256, 1L << 20)); }

std::vector<AuxFn> expand(const rid_aux_basis_desc& d) {
  struct Sh { int atom, l; double e; };
  std::vector<Sh> shells;
  if (d.nshell > 0) {
    for (int s = 0; s < d.nshell; ++s) shells.push_back(Sh{d.shell_atom_host[s], d.shell_l_host[s], d.shell_exp_host[s]});
  } else {
    for (int a = 0; a < d.natom; ++a)
      for (int l = 0; l <= d.lmax; ++l) shells.push_back(Sh{a, l, d.theta / (d.radius_host[a] * d.radius_host[a])});
  }
  std::vector<AuxFn> out;
  for (int l = 0; l <= 2; ++l)
    for (const Sh& s : shells) {
      if (s.l != l) continue;
      const double* c = d.coords_host + 3L * s.atom;
      const int first = l == 0 ? 0 : (l == 1 ? 1 : 4), cnt = l == 0 ? 1 : (l == 1 ? 3 : 5);
      for (int k = 0; k < cnt; ++k) out.push_back(AuxFn{c[0], c[1], c[2], s.e, first + k, 0});
    }
  return out;
}

}  // namespace

void aux_basis_check(const rid_aux_basis_desc& d) {
  RID_CHECK(d.natom >= 1 && d.coords_host && d.ao_count_host && d.ao_exp_host, RID_ERR_INVALID_ARG,
            "molecule: atoms, coordinates and atomic orbitals are required");
  RID_CHECK(d.no >= 1 && d.nv >= 1 && d.nao >= d.no + d.nv, RID_ERR_SHAPE,
            "molecule: need no, nv >= 1 and at least no + nv atomic orbitals");
  long nao = 0;
  for (int a = 0; a < d.natom; ++a) {
    RID_CHECK(d.ao_count_host[a] >= 0, RID_ERR_INVALID_ARG, "negative atomic-orbital count");
    nao += d.ao_count_host[a];
  }
  RID_CHECK(nao == d.nao, RID_ERR_SHAPE, "ao_count does not add up to nao");
  for (long m = 0; m < nao; ++m)
    RID_CHECK(d.ao_exp_host[m] > 0.0 && std::isfinite(d.ao_exp_host[m]), RID_ERR_INVALID_ARG, "bad AO exponent");
  RID_CHECK(d.kappa > 0.0 && std::isfinite(d.kappa), RID_ERR_INVALID_ARG, "kappa must be > 0");
  if (d.nshell > 0) {
    RID_CHECK(d.shell_atom_host && d.shell_l_host && d.shell_exp_host, RID_ERR_INVALID_ARG, "shell arrays missing");
    for (int s = 0; s < d.nshell; ++s) {
      RID_CHECK(d.shell_atom_host[s] >= 0 && d.shell_atom_host[s] < d.natom, RID_ERR_INVALID_ARG, "shell atom");
      RID_CHECK(d.shell_l_host[s] >= 0 && d.shell_l_host[s] <= 2, RID_ERR_INVALID_ARG, "shells must have l <= 2");
      RID_CHECK(d.shell_exp_host[s] > 0.0 && std::isfinite(d.shell_exp_host[s]), RID_ERR_INVALID_ARG,
                "bad shell exponent");
    }
  } else {
    RID_CHECK(d.radius_host && d.theta > 0.0 && d.lmax >= 0 && d.lmax <= 2, RID_ERR_INVALID_ARG,
              "the exponent rule needs radii, theta > 0 and 0 <= lmax <= 2");
    for (int a = 0; a < d.natom; ++a) RID_CHECK(d.radius_host[a] > 0.0, RID_ERR_INVALID_ARG, "radius must be > 0");
  }
}

void aux_basis_size(const rid_aux_basis_desc& d, int* naux, int* naux_s) {
  aux_basis_check(d);
  const std::vector<AuxFn> f = expand(d);
  RID_CHECK(f.size() <= (size_t)kMaxProjected, RID_ERR_SHAPE,
            "auxiliary basis above 1024 functions (the metric is factored in one workgroup)");
  *naux = (int)f.size();
  int s = 0;
  for (const AuxFn& x : f) s += x.kind == 0;
  *naux_s = s;
}

void aux_tensor_build(rid_context* ctx, const rid_aux_basis_desc& d, double* bia, double* bij, double* bab) {
  int naux = 0, ns = 0;
  aux_basis_size(d, &naux, &ns);
  RID_CHECK(d.mo_dev && bia && bij && bab, RID_ERR_INVALID_ARG, "null device pointer");
  hipStream_t st = ctx->stream;
  const std::vector<AuxFn> fn = expand(d);
  const int nao = d.nao, nmo = d.no + d.nv;
  // atomic orbitals: centre, exponent, normalisation (2a/pi)^(3/4)
  std::vector<double> ao(5L * nao);
  {
    long m = 0;
    for (int a = 0; a < d.natom; ++a)
      for (int k = 0; k < d.ao_count_host[a]; ++k, ++m) {
        const double e = d.ao_exp_host[m];
        ao[5 * m + 0] = d.coords_host[3 * a + 0];
        ao[5 * m + 1] = d.coords_host[3 * a + 1];
        ao[5 * m + 2] = d.coords_host[3 * a + 2];
        ao[5 * m + 3] = e;
        ao[5 * m + 4] = std::pow(2.0 * e / M_PI, 0.75);
      }
  }
  DevBuf dfn(ctx), dao(ctx), J(ctx), G(ctx), info(ctx), X(ctx), Ct(ctx), T(ctx), K(ctx), Kt(ctx), B(ctx);
  dfn.ensure(sizeof(AuxFn) * fn.size());
  dao.ensure(sizeof(double) * ao.size());
  RID_HIP(hipMemcpyAsync(dfn.p, fn.data(), sizeof(AuxFn) * fn.size(), hipMemcpyHostToDevice, st));
  RID_HIP(hipMemcpyAsync(dao.p, ao.data(), sizeof(double) * ao.size(), hipMemcpyHostToDevice, st));
  // metric and its Cholesky factor and inverse
  J.ensure(sizeof(double) * (size_t)naux * naux);
  G.ensure(sizeof(double) * (size_t)naux * naux);
  info.ensure(sizeof(int));
  hipLaunchKernelGGL(metric_kernel, dim3(grid_of((long)naux * naux)), dim3(256), 0, st, dfn.as<AuxFn>(), naux,
                     J.as<double>());
  RID_HIP(hipGetLastError());
  small_chol(J.as<double>(), naux, naux, info.as<int>(), st);
  int ok = 0;
  RID_HIP(hipMemcpyAsync(&ok, info.p, sizeof(int), hipMemcpyDeviceToHost, st));
  RID_HIP(hipStreamSynchronize(st));
  RID_CHECK(ok == 0, RID_ERR_INDEFINITE, "auxiliary metric (P|Q) is not positive definite");
  small_trinv_lower(J.as<double>(), naux, naux, G.as<double>(), naux, st);
  // three-centre integrals over atomic orbitals
  X.ensure(sizeof(double) * (size_t)naux * nao * nao);
  hipLaunchKernelGGL(three_center_kernel, dim3(grid_of((long)naux * nao * nao)), dim3(256), 0, st, dao.as<double>(),
                     nao, dfn.as<AuxFn>(), naux, X.as<double>());
  RID_HIP(hipGetLastError());
  // K[P] = C^T X[P] C in two products over the batch of P: with Ct = C^T
  // (nmo x nao), T[P] = Ct X[P] (nmo x nao, X[P] symmetric), K[P] = Ct T[P]^T
  Ct.ensure(sizeof(double) * (size_t)nmo * nao);
  transpose_slices<double, double>(d.mo_dev, 1, nao, nmo, Ct.as<double>(), st);
  T.ensure(sizeof(double) * (size_t)naux * nmo * nao);
  K.ensure(sizeof(double) * (size_t)naux * nmo * nmo);
  {
    GemmParams g{};
    g.A = Ct.p;
    g.B = X.p;
    g.C = T.p;
    g.M = nmo;
    g.N = nao;
    g.K = nao;
    g.np = 1;
    g.pps = 1;
    g.nz2 = 1;
    g.lda = nao;
    g.ldb = nao;
    g.ldc = nao;
    g.sA1 = 0;
    g.sB1 = (long)nao * nao;
    g.sC1 = (long)nmo * nao;
    g.alpha = 1.0;
    g.mode = GEMM_STORE;
    g.order = ORDER_MN;
    gemm_nt<double>(g, naux, 1, st);
    GemmParams h = g;
    h.B = T.p;
    h.C = K.p;
    h.N = nmo;
    h.ldb = nao;
    h.ldc = nmo;
    h.sB1 = (long)nmo * nao;
    h.sC1 = (long)nmo * nmo;
    gemm_nt<double>(h, naux, 1, st);
  }
  X.release();
  T.release();
  // B = sqrt(kappa) G K over (p, q), with K read transposed (K-contiguous)
  const long npq = (long)nmo * nmo;
  Kt.ensure(sizeof(double) * (size_t)npq * naux);
  transpose_slices<double, double>(K.as<double>(), 1, naux, (int)npq, Kt.as<double>(), st);
  K.release();
  B.ensure(sizeof(double) * (size_t)npq * naux);
  {
    GemmParams g{};
    g.A = G.p;
    g.B = Kt.p;
    g.C = B.p;
    g.M = naux;
    g.N = (int)npq;
    g.K = naux;
    g.np = 1;
    g.pps = 1;
    g.nz2 = 1;
    g.lda = naux;
    g.ldb = naux;
    g.ldc = npq;
    g.alpha = std::sqrt(d.kappa);
    g.mode = GEMM_STORE;
    g.order = ORDER_MN;
    gemm_nt<double>(g, 1, 1, st);
  }
  hipLaunchKernelGGL(split_blocks_kernel, dim3(grid_of(npq * naux)), dim3(256), 0, st, B.as<double>(), naux, d.no,
                     d.nv, bia, bij, bab);
  RID_HIP(hipGetLastError());
  RID_HIP(hipStreamSynchronize(st));
}

}  // namespace rid

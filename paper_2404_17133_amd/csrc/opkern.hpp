// Memory-bound kernels around the operator contractions (see opkern.hip).
#pragma once

#include "common.hpp"

namespace rid {

struct CombineArgs {
  const double* x;   // nvec x N input vectors (f64)
  const double* de;  // N: eps_a - eps_i
  const double* j;   // nvec x N Coulomb product sum_P B^P_ia t^P (or null)
  double* y;         // output (A x, T x, or (A+B) x in pair mode)
  double* y2;        // pair mode: (A-B) x
  int nvec, no, nv;
  int i0, no_a, nv_a; // exchange window
  int ns_w, ns_wp;    // split counts of the W and W' partials
  long sstride;       // stride between splits of the partials
  double cj;          // Coulomb factor: 2 (A, T) or 4 (A+B, T+)
  double a_x;
  int pair;
};

template <typename E>
void prep_x(const double* x, int nvec, int no, int nv, int i0, int no_a, int nv_a, int kv, E* xc, E* xa, E* xt,
            hipStream_t s);
template <typename A>
void reduce_splits(const A* part, int ns, long stride, long n, double* out, hipStream_t s);
template <typename E>
void coul_bwd(const double* t, const E* b, int naux, long n, int nvec, double* j, double* part, size_t part_elems,
              hipStream_t s);
// Ranges of the auxiliary index coul_bwd splits into (its partial buffer
// holds that many nvec x n blocks; with less it runs unsplit).
int coul_bwd_splits(long n, int nvec, int naux);
template <typename A>
void combine(const CombineArgs& c, const A* wp, const A* wpp, hipStream_t s);
template <typename S, typename E>
void cast_copy(const S* src, long n, E* dst, hipStream_t s);
template <typename S, typename E>
void transpose_slices(const S* src, int np, int rows, int cols, E* dst, hipStream_t s);

}  // namespace rid

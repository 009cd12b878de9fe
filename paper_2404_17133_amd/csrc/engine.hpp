// Krylov solvers of the library (see engine.hip).
#pragma once

#include <vector>

#include "core.hpp"

namespace rid {

struct SolveStats {
  int n_iter = 0, n_mv = 0, n_inner_mv = 0, n_inner_iter = 0;
  int n_blocks_cholqr = 0, n_blocks_mgs = 0;  // orthonormalisation routes taken
  std::vector<double> history;
  double t_matvec = 0.0, t_precond = 0.0, t_other = 0.0, t_total = 0.0;  // ms
  uint64_t peak_bytes = 0;
};

// The public statistics of a solve (zeroes out first; out may be null).
void fill_stats(rid_stats* out, const SolveStats& s);

// Where a solve runs: its stream (null: the context stream) and, for solves
// that share the device with others, the Batcher that groups their operator
// products (null: products run directly on the solve's stream with the
// problem's scratch).
struct ExecCfg {
  hipStream_t stream = nullptr;
  Batcher* batcher = nullptr;
};

// k lowest roots; TDA (mode 0) or full TDDFT (mode 1).  Returns RID_OK,
// RID_WARN_NOT_CONVERGED or throws rid::Error.
rid_status eigen_solve(rid_problem* P, const rid_solve_opts& o, int k, int mode, double* omega_host, double* x_dev,
                       double* y_dev, double* resid_host, SolveStats& st, const ExecCfg& ex = ExecCfg());

rid_status response_solve(rid_problem* P, const rid_solve_opts& o, int nrhs, const double* p_dev, int nfreq,
                          const double* omega_host, double* alpha_host, double* u_dev, double* resid_host,
                          SolveStats& st, const ExecCfg& ex = ExecCfg());

void validate_opts(const rid_solve_opts& o, const rid_problem* P);

}  // namespace rid

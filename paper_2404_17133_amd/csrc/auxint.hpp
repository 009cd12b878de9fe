// Auxiliary-basis RI tensors built from a molecule (see auxint.hip).
#pragma once

#include "core.hpp"

namespace rid {

void aux_basis_check(const rid_aux_basis_desc& d);
// Number of auxiliary functions, and of s functions (the leading rows).
void aux_basis_size(const rid_aux_basis_desc& d, int* naux, int* naux_s);
// B^P_ia, B^P_ij, B^P_ab (FP64, caller's device buffers) on the context stream; synchronous.
void aux_tensor_build(rid_context* ctx, const rid_aux_basis_desc& d, double* bia, double* bij, double* bab);

}  // namespace rid

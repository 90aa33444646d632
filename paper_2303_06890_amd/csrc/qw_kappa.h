// Host computation of the smallest eigenvalue magnitude of A/s for the CKS
// schedule (qw_kappa.cpp).  Not part of the public ABI.
#pragma once

#include <stdint.h>

#include <string>

namespace qw {

// min |lambda| of A/s for one instance: n = unpadded dimension, s = slots per
// row, nbits = log2 of the padded dimension, col/val = the row-major QRAM
// table of the instance (slot (j, l) at j*s + l; val holds each slot's
// rotation angle when `angles`), vim_home = imaginary parts by home
// (l << nbits) + j, or NULL.  Returns 0, or -1 (QW_EINVAL: singular matrix,
// entry outside the matrix) / -5 (QW_ENOTSUP: not symmetric or Hermitian,
// iteration not converged) with the reason in err.
int min_abs_eigenvalue(int32_t n, int32_t s, int32_t nbits, const int32_t* col, const double* val,
                       const double* vim_home, bool angles, double* lam, std::string& err);

}  // namespace qw

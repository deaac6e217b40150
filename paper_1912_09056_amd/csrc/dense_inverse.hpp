// Device inverse of a dense FP64 matrix (blocked LU with partial pivoting,
// FP64 matrix-core updates): the coarsest-level direct solve's setup.
#pragma once

#include "common.hpp"

namespace camg {

// a: device, row-major n x n FP64.  Writes A^-1 row-major to inv and its
// transpose row-major to invT (either may be null), rounded to T.  A pivot
// not above `tiny` (partial pivoting: largest magnitude, first row on ties)
// returns false and leaves the outputs undefined.  Allocates a padded
// workspace of two (n rounded up to 64)^2 FP64 matrices; synchronises s.
template <typename T>
bool dense_inverse(const double* a, int64_t n, double tiny, T* inv, T* invT, hipStream_t s);

// out[0] (device) = max |a_e| over the n entries of the device array a, NaN
// when one is not finite.  Asynchronous.
void max_abs(const double* a, int64_t n, double* out, hipStream_t s);

}  // namespace camg

// Host side of the DAXPY kernel (y <- alpha*x + y).
#pragma once

#include "common.h"

namespace mg {

// Enqueues y[i*incy] <- fma(alpha, x[i*incx], y[i*incy]) for i < n
// (arguments already validated: incx, incy >= 1; alpha == 0 or n == 0 is a
// no-op).
int axpy_f64(int64_t n, double alpha, const double *x, int64_t incx, double *y, int64_t incy,
             hipStream_t s);

}  // namespace mg

/*
 * Algorithm-matched CPU baseline: cell-list LJ molecular dynamics on the
 * host cores (OpenMP threads, SIMD pair loops), in FP32 (cc_run_f32) and FP64
 * (cc_run_f64). It is a
 * performance reference for the GPU library, independent of it and of the
 * brute-force oracle; a test pins its forces to the oracle's.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct cc_params {
    double box, epsilon, sigma, rc, mass, dt;
} cc_params;

int cc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void cc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

#define REAL float
#define FLOOR floorf
#define SQRT sqrtf
#define NAME(x) cc_##x##_f32
#include "cells_cpu_impl.h"
#undef REAL
#undef FLOOR
#undef SQRT
#undef NAME

#define REAL double
#define FLOOR floor
#define SQRT sqrt
#define NAME(x) cc_##x##_f64
#include "cells_cpu_impl.h"
#undef REAL
#undef FLOOR
#undef SQRT
#undef NAME

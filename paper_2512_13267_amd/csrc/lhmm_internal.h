// lhmm_internal.h -- helpers shared by the library's translation units (not
// part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include "lhmm.h"

// Record a thread-local error message for lhmm_last_error(); returns code.
int lhmm_fail(int code, const char* fmt, ...);
// Clear the thread-local error message.
void lhmm_clear_error();
// The caller stream a micro engine was created with.
hipStream_t lhmm_micro_caller_stream(const lhmm_micro* m);
// The stream an SPH engine launches on, its particle count and mobile count.
hipStream_t lhmm_sph_caller_stream(const lhmm_sph* s);
void lhmm_sph_counts(const lhmm_sph* s, int* n, int* n_mobile);
// The stream of a surrogate engine and its dimensions.
hipStream_t lhmm_sur_caller_stream(const lhmm_sur* s);
void lhmm_sur_dims(const lhmm_sur* s, int* n_members, int* n_in, int* n_out, int* max_batch);

#define LHMM_HIPCHK(expr)                                                                        \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess) return lhmm_fail(LHMM_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

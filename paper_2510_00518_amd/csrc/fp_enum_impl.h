// Internal interface of the host enumerator (fp_enum.cpp) for the library's
// streaming executor: one row at a time, with a record window, so a row longer
// than a streaming chunk can be produced piece by piece.  Not part of the C ABI.
#pragma once

#include <cstdint>
#include <functional>

#include "fp.h"

namespace fpenum {

struct Handle;

// Same rules as fp_enumerate_count/fill with keep_fraction 1.  The arrays are
// borrowed, not copied: they must outlive the handle.
fp_status open(Handle** h, int32_t type, const int32_t mesh[3], int32_t nb, const double* omega,
               double omega_floor, double sigma, double nsigma, const double* vel, const fp_broadening* br);
void close(Handle* h);

// Number of records of row g0 (a valid global mode index).
int64_t count_row(const Handle* h, int32_t g0);

// Records [begin, end) of row g0, in the enumerator's order, written to out;
// returns how many were written (end - begin unless the row is shorter).
int64_t fill_row(const Handle* h, int32_t g0, int64_t begin, int64_t end, uint64_t* out);

// body(i) for every i in [0, n) on up to n_threads host threads (<= 0: every
// hardware thread); i is handed out by an atomic counter.
void parallel_for(int64_t n, int32_t n_threads, const std::function<void(int64_t)>& body);

}  // namespace fpenum

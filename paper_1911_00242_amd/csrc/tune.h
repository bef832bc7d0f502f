// Measurements for the choice of arithmetic form per mixed-precision product (tune.cpp).
#pragma once
#include <string>
#include <vector>

#include "common.h"
#include "mixed.h"

namespace ck {

// What was measured for one product shape: average launch time (ms) of each arithmetic form
// on the system's own operands and tables, and each form's error on seeded operands.
struct TuneRecord {
    double ms[ARITH_COUNT] = {};
    double err[ARITH_COUNT] = {};
};

// max |C_form - C_fp64| / max |C_fp64| of each arithmetic form on one seeded M x N x K
// product (complex operands with standard normal parts), against the FP64 MFMA kernel.
std::vector<double> form_errors(int M, int N, int K, uint64_t seed, hipStream_t st);
// "<device name>/<gfx arch>" of the current device
std::string device_key();
std::string tune_key(const std::string &dev, int G, int M, int N, int K, int fast);
// text cache, one record per line: key, ARITH_COUNT times, ARITH_COUNT errors
bool cache_lookup(const char *path, const std::string &key, TuneRecord &out);
void cache_store(const char *path, const std::string &key, const TuneRecord &r);

}  // namespace ck

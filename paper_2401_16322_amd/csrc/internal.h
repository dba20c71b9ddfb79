// Internal declarations shared by the host-math and device parts of the library.
#pragma once

#include <cstdarg>
#include <cstdint>
#include <string>
#include <vector>

#include "expwave.h"

namespace expw {

// Sets the thread-local message returned by expw_last_error() and returns code.
int32_t fail(int32_t code, const char* fmt, ...);
void clear_error();

// Staggered first-derivative weights alpha_1..alpha_K (Sec. 2.1); K = order/2.
bool stagger_weights(int order, double* alpha /* >= 4 entries */, int* K);

// Host math (FP64).
void damping_profile(int64_t n, double h, int cells, double sigma_max, bool half, double* out);
void faber_coefficients(double gamma, double c0, double c1, double dt, int m, double* a);
void ricker_derivatives(double t, double f_peak, double t_delay, int p, double* out);
void faber_source_scalars(double gamma, double c0, double c1, int m, int p, const double* G,
                          double* q);
bool expm(int k, const double* A, double* E);
// The ellipse a Faber step in state precision dtype runs with: 1/gamma, c0
// and c1 rounded to that precision, gamma taken back from the rounded 1/gamma.
void step_ellipse(int dtype, double gamma, double c0, double c1, double* gs, double* c0s,
                  double* c1s);

}  // namespace expw

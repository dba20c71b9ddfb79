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
// The staggered weights as alpha_l = beta * w_l with small integers w_l
// (exact in FP32).
bool stagger_weights_int(int order, double* w /* >= 4 entries */, double* beta, int* K);

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
// PML operator: Fornberg weights (c[k * n + i], derivative orders 0..m), the
// free-surface tables, and beta_y (layer at the bottom only).
void fd_weights(double z0, const double* nodes, int n, int m, double* c);
void pml_surface_tables(double d2[4][9], double d1[3][8], double dw[4][8]);
void bottom_profile(int64_t n, double h, int cells, double beta0, bool half, double* out);

}  // namespace expw

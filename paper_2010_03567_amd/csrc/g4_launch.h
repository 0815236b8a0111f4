// g4_launch.h -- host-side launchers and helpers of the HIP sources of
// libg4hip.so (not part of the public ABI); included by g4_internal.h after
// the data layout it refers to.
#pragma once

// phase k of the timers: 0 build, 1 moments, 2 seed, 3 walk
int g4_phase_begin(g4_ctx *ctx, g4_tree *t, int k);
int g4_phase_end(g4_ctx *ctx, g4_tree *t, int k);
// seconds between the recorded events of phase k (0 if not recorded); the
// events must be complete (the caller has synchronised the stream)
double g4_phase_seconds(const g4_tree *t, int k);

// host launchers implemented in the .hip files
int g4_launch_build(g4_ctx *ctx, g4_tree *t, const g4_particles *p);
int g4_launch_moments(g4_ctx *ctx, g4_tree *t);
int g4_launch_build_forest(g4_ctx *ctx, g4_tree *t, const g4_particles *p, const int64_t *off_dev, uint32_t *bkey0,
                           uint32_t *bkey1);
int g4_launch_walk(g4_ctx *ctx, g4_tree *t, const g4_walk_params *wp, int kernel, int criterion,
                   double *ax, double *ay, double *az, double *pot, uint32_t *counts, float *aout_caller,
                   float *aout_sorted, int stat_slot, bool count);
int g4_launch_export(g4_ctx *ctx, const g4_tree *t, int32_t *level, uint32_t *cell, int64_t *count,
                     int64_t *first, int32_t *leaf, double *mass, double *com, double *q2, double *q3);
int g4_launch_direct(g4_ctx *ctx, const g4_particles *p, const g4_tree_params *tp, const g4_walk_params *wp,
                     int truncate, const int64_t *targets, int64_t ntargets, double *ax, double *ay, double *az,
                     double *pot);
int g4_launch_quantize(g4_ctx *ctx, const double *pos, int64_t n, const g4_tree_params *tp, uint32_t *x,
                       uint32_t *y, uint32_t *z, int32_t *flag);
int g4_launch_gather_seed(g4_ctx *ctx, g4_tree *t, const float *a_seed_caller);
// stable LSD radix sort of (key, value) pairs over bits [bit_lo, bit_hi) in
// 8-bit digits, ping-ponging between (k0, v0) and (k1, v1); *in_alt = 1 when
// the sorted pairs end in (k1, v1), 0 when in (k0, v0).  temp: device bytes of
// g4_radix_sort_temp_bytes(n).  Enqueued on the context's stream.
size_t g4_radix_sort_temp_bytes(int64_t n);
int g4_radix_sort_u64(g4_ctx *ctx, uint64_t *k0, uint64_t *k1, uint32_t *v0, uint32_t *v1, int64_t n, int bit_lo,
                      int bit_hi, void *temp, size_t temp_bytes, int *in_alt);
int g4_radix_sort_u32(g4_ctx *ctx, uint32_t *k0, uint32_t *k1, uint32_t *v0, uint32_t *v1, int64_t n, int bit_lo,
                      int bit_hi, void *temp, size_t temp_bytes, int *in_alt);
// zero `bytes` (a multiple of 4) of device memory with a kernel, so that the
// calls stay valid under stream capture (no memset nodes in a graph)
int g4_launch_zero(g4_ctx *ctx, void *p, size_t bytes);
int g4_launch_mlp_features(g4_ctx *ctx, const g4_tree *t, const g4_walk_params *wp, const float *norm,
                           float *feat);
int g4_launch_mlp_forward(g4_ctx *ctx, const uint16_t *w, const float *feat, int64_t n, float *out, float shift,
                          int mode);
int g4_launch_mlp_grad(g4_ctx *ctx, const uint16_t *w, const float *feat, const float *target, int64_t n,
                       float tau, float *grad, float *loss);
int g4_pm_layout_bytes(int ng, size_t *bytes);
int g4_launch_pm(g4_ctx *ctx, const g4_tree *t, const g4_pm_params *pp, void *ws, size_t ws_bytes, int accumulate,
                 double *ax, double *ay, double *az, double *pot);
int g4_fmm_layout_bytes(const g4_tree *t, const g4_fmm_params *fp, double factor, size_t *bytes);
int g4_launch_fmm(g4_ctx *ctx, g4_tree *t, const g4_fmm_params *fp, double factor, void *ws, size_t ws_bytes,
                  double *ax, double *ay, double *az, double *pot, g4_stats *stats);
int g4_launch_mlp_adam(g4_ctx *ctx, uint16_t *w, float *master, float *m, float *v, const float *grad, float lr,
                       float b1, float b2, float eps, int64_t step);
int g4_kdk_layout_bytes(const g4_kdk_params *kp, int64_t n, size_t *bytes);
int g4_launch_kdk(g4_ctx *ctx, const g4_kdk_params *kp, int64_t n, double *pos, double *vel, const float *mass,
                  double dt, double *ax, double *ay, double *az, int have_acc, void *ws, size_t ws_bytes,
                  g4_kdk_stats *stats);
size_t g4_ewald_layout_bytes(int ne);
int g4_launch_ewald_table(g4_ctx *ctx, double box, int ne, float *tab);
int g4_launch_ewald_eval(g4_ctx *ctx, const float *tab, int ne, double box, int64_t n, const double *dx,
                         const double *dy, const double *dz, double *psi, double *gx, double *gy, double *gz);
int g4_launch_moments4(g4_ctx *ctx, g4_tree *t, double *q4);

// Internal interface of the learned scorer (not part of the C-ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/skyline.h"

int sky_ctx_device(const sky_ctx *c);
int sky_mlp_dim(const sky_mlp *m);
// Unique per model created in the process (never reused): captured graphs that
// bake a model's buffers are keyed by it.
uint64_t sky_mlp_serial(const sky_mlp *m);
// Scores of n points into out (device), on stream s. Returns a SKY_* code.
int sky_mlp_score_internal(const sky_mlp *m, const float *pts, uint32_t n, int d, float *out, hipStream_t s);
// Looks up, with `device` current, the device address of the scratch array that
// sky_mlp_targets_noalloc uses on that device (once per device; later calls
// return at once). Returns a SKY_* code.
#define SKY_MAX_DEVICES 64
int sky_noalloc_setup(int device);

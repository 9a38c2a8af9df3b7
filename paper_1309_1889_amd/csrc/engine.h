// Internal interface between the engine and the integrator translation units.
#pragma once

#include <hip/hip_runtime.h>

struct msm_ctx;

int msmx_ctx_precision(const msm_ctx *c);
hipStream_t msmx_ctx_stream(const msm_ctx *c);

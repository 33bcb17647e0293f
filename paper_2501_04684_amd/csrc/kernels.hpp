// Launchers of the far-zone kernels (defined in kernels.hip). Each one only
// enqueues work on `stream` (a hipStream_t) and returns the hipError_t of
// the launch as an int (0 = success).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

#include "plan.hpp"

namespace ubf {

// Optional timing of one stage: the kernel's own dispatch records `start`
// when it begins and `stop` when it ends (hipExtLaunchKernel), so their
// elapsed time is the kernel's execution alone, with no marker between
// kernels. A stage that launches nothing records both on the stream.
struct StageEvents {
  hipEvent_t start;
  hipEvent_t stop;
};

// Identity basis: complex [nrhs][n_box][nu] -> planar padded box vectors.
int launch_pack(const Plan& p, const void* x, float* P, int nrhs, void* stream,
                const StageEvents* ev = nullptr);

// Planar padded box vectors -> complex [nrhs][n_box][nu].
int launch_unpack(const Plan& p, const float* P, void* out, int nrhs, void* stream);

// Stage 1: P_i = S_i x_i (planar padded output).
int launch_aggregate(const Plan& p, const void* x, float* P, int nrhs, void* stream,
                     const StageEvents* ev = nullptr);

// Stage 2: per-pair products G_w P_src into the partial buffer.
int launch_translate(const Plan& p, const float* P, float* part, int nrhs,
                     void* stream, const StageEvents* ev = nullptr);

// Stage 3: y_j = T_j E_j, where E_j is either the sum of the test box's
// partial products (from_parts) or read from a complex vector `E`.
// `identity` forces y_j = E_j whatever basis the plan holds.
int launch_disaggregate(const Plan& p, bool from_parts, const float* part,
                        const void* E, void* y, int nrhs, void* stream,
                        bool identity = false, const StageEvents* ev = nullptr);

// True if stage 2 for this plan runs on the matrix cores.
bool translate_uses_mfma(const Plan& p);

}  // namespace ubf

// Network translation (Sec. 3): shapes, the device image of a plan's
// networks and the launchers (networks.hip). Each launcher only enqueues
// work and returns the hipError_t of the launch as an int (0 = success).
#pragma once

#include <cstddef>

#include "kernels.hpp"
#include "plan.hpp"

namespace ubf {

constexpr int kMaxHidden = 64;  // hidden units per network

// Box sizes with a network kernel (3 n_d^3 for n_d = 2, 3, 4) and widths.
bool network_shape_supported(int nu, int hidden);

// Hidden units per part in the image: the width rounded up to 32.
int network_hp(int hidden);

// Bytes of the device image of one network per offset of the plan.
size_t network_image_bytes(const Plan& p, int hidden);

// Caller weights (complex64, offsets in plan order: W1 [n_off][H][nu],
// b1 [n_off][H], W2 [n_off][nu][H], b2 [n_off][nu]) -> image `img`.
int launch_network_pack(const Plan& p, int hidden, const void* W1, const void* b1,
                        const void* W2, const void* b2, float* img, void* stream);

// Stage 2 with the plan's networks: per-pair network products (each source
// box vector scaled by its own l-inf norm) into the partial rows.
int launch_translate_cvfcnn(const Plan& p, const float* P, float* part, int nrhs, void* stream,
                            const StageEvents* ev = nullptr);

// Stage 2 by the FP32 operator table with the box vectors staged in LDS,
// for box sizes whose columns do not fit in registers (N_u = 192).
bool staged_translate_supported(const Plan& p);
int launch_translate_staged(const Plan& p, const float* P, float* part, int nrhs, void* stream,
                            const StageEvents* ev = nullptr);

}  // namespace ubf

// Seeder constants shared by the host runtime and the kernels.
#pragma once

#include <cstddef>

namespace mu {

constexpr int kSeedLayers = 4;   // 1024-512-256-128-8
constexpr int kSeedUsedOut = 5;  // outputs with a loss weight: A, log lambda, log nu, cos phi, sin phi
size_t seeder_param_count();

}  // namespace mu

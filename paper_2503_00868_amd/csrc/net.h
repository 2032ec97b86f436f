// Learned preconditioner (3-level 3-D U-Net) used inside flexible CG.
#pragma once

#include <stddef.h>

#include "ctx.h"

namespace fs {

size_t net_workspace_bytes(int n);
int net_init(sim_ctx* c);
void net_destroy(sim_ctx* c);
bool net_ready(const sim_ctx* c);
// z = mask * rms(r) * U(r / rms(r), mask); returns at once when flags (nullable)
// has the done flag raised.
int net_apply(sim_ctx* c, const float* r, float* z, const int* flags);

}  // namespace fs

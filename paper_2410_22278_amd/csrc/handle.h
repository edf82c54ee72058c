// Internal C++ interface to a pbc_jk handle, used by the request server:
// host setup and device creation are separate steps so that a request's
// device footprint is known before it is admitted.
#pragma once
#include <cstddef>

#include "arena.h"
#include "pbcjk.h"

namespace pbcjk {

// Host setup only (validation, pair and G lists); no device memory.
int handle_new(const pbc_cell *cell, const pbc_atoms *atoms, const pbc_basis *basis, double omega,
               const pbc_jk_thresholds *thr, pbc_jk **out);
// Device bytes of the setup data and work buffers (everything except the
// real-space neighbour lists), as the allocator would round them.
size_t handle_fixed_bytes(pbc_jk *h, double lr_budget_mb);
// Uploads the setup data, allocates the work buffers and builds the
// neighbour lists, from `arena` (NULL = hipMalloc).  On failure the device
// part is released and the host setup kept (the call may be repeated).
int handle_device(pbc_jk *h, Arena *arena, bool profile, double lr_budget_mb);
// Releases the device part only.
void handle_drop_device(pbc_jk *h);
// Neighbour-list bytes, known once handle_device has counted them (else 0).
size_t handle_nbr_bytes(const pbc_jk *h);
size_t handle_dev_bytes(const pbc_jk *h);
int handle_natom(const pbc_jk *h);
void handle_delete(pbc_jk *h);

}  // namespace pbcjk

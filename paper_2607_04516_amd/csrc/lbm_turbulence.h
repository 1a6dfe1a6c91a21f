// Synthetic von Karman inflow generator (App. F): internal interface
// between the C-ABI runtime and lbm_turbulence.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "lbm.h"
#include "lbm_device.h"

namespace lbm {

struct VkGen;

// Build the generator for one grid: active cells from the geometry, the host
// copy of the solid bits ([nz][ny][wpr] words) and the per-cell boundary
// states (host [n_in][3] by inflow_slot: each cell's mean velocity U_b),
// mode tables from the parameters; device buffers allocated here.  Returns
// an LBM_* code; err holds the message.
int vk_create(VkGen** out, const lbm_turbulence& p, const Geo& g, const std::vector<uint64_t>& bits,
              const std::vector<double>& base, std::string& err);
void vk_destroy(VkGen* v);

// Make uin (device per-cell inflow velocities) hold U(t) at the active
// cells, evaluating the series only at new anchors when a stride is set.
hipError_t vk_apply(VkGen* v, double* uin, int64_t t, hipStream_t s);

// Forget cached anchors (uin was rewritten from the boundary states).
void vk_invalidate(VkGen* v);

void vk_info(const VkGen* v, int64_t* n_active, double* u_ref, double* e_c);

}  // namespace lbm

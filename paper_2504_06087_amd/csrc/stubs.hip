// Workspace sizing across entry points.
#include "laplacian.hpp"
#include "update.hpp"
#include "paths.hpp"
namespace fire {
size_t grad_ws_bytes(const fire_handle* h, int W);
size_t workspace_bytes_for(const fire_handle* h, int W) {
  const size_t v[8] = {ws_forward(h, W).total, upd_layout(h, W).total, lap_ws_bytes(h, W), ecp_ws_bytes(h, W),
                       grad_ws_bytes(h, W), rng_ws_offset(h, W) + rng_ws_bytes(h, W), spring_ws_bytes(h->P, W),
                       swap_ws_bytes(h, W)};
  size_t m = 0;
  for (size_t x : v) m = x > m ? x : m;
  return m;
}
}  // namespace fire

// Workspace sizing across entry points and the parameter-gradient entry (adjoint).
#include "laplacian.hpp"
#include "update.hpp"
namespace fire {
size_t workspace_bytes_for(const fire_handle* h, int W) {
  size_t a = ws_forward(h, W).total, b = upd_layout(h, W).total, c = lap_ws_bytes(h, W), d = ecp_ws_bytes(h, W);
  size_t m = a > b ? a : b;
  m = m > c ? m : c;
  return m > d ? m : d;
}
hipError_t grad_path(fire_handle*, int, const double*, char*, char*, const double*, double*, int32_t*,
                     hipStream_t) { return hipErrorNotSupported; }
}

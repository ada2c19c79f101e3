// Host-side launch interface of the compact panel kernels (panel.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "k_gj.hpp"

namespace hss {

struct PanelShape {
  int nb, rpt, nt;  // panel width, rows per thread, threads per workgroup
};

// Shape of the compact panel kernel for panels of at most `rows` rows; false when
// no instantiation holds that many rows in registers.
template <class X> bool panel_rot_config(int rows, PanelShape& s);

// Launch gj_panel_rot_kernel for nn boxes (descriptors on the device).
template <class X>
void launch_panel_rot(const GjDesc<X>* dd, int nn, int j0, int nb, const PanelShape& s, hipStream_t st);

}  // namespace hss

// Host-side launch interface of the compact panel kernels (panel.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "k_gj.hpp"

namespace hss {

struct PanelShape {
  int nb, rpt, nt;  // panel width, rows per thread, threads per workgroup
};

// Shape of the compact panel kernel for panels of at most `rows` rows; false when
// no instantiation holds that many rows in registers.
template <class X> bool panel_rot_config(int rows, PanelShape& s);

// Whether a compact panel of shape s is compiled for X.
template <class X> bool panel_rot_compiled(const PanelShape& s);

// Launch gj_panel_rot_kernel for nn boxes (descriptors on the device).
template <class X>
void launch_panel_rot(const GjDesc<X>* dd, int nn, int j0, int nb, const PanelShape& s, hipStream_t st);

// Tournament pivoting for panels above the compact kernels' capacity: the width
// (16), the chunk of rows each local search holds in registers (tourn_chunk: four
// rows per thread, two for complex128, whose values take four registers each) and
// the largest number of candidate rows of the final search (tourn_cand).
template <class X> constexpr int tourn_nb() { return 16; }
template <class X> constexpr int tourn_rpt() { return std::is_same<X, cd>::value ? 2 : 4; }
template <class X> constexpr int tourn_chunk() { return 256 * tourn_rpt<X>(); }
template <class X> constexpr int tourn_cand() { return std::is_same<X, cd>::value ? 512 : 256; }

// Launch the local searches (grid nch x nn) and the final search (grid nn) of one
// panel step; cand holds nn * nch * tourn_nb<X>() ints.
template <class X>
void launch_panel_tourn(const GjDesc<X>* dd, int nn, int j0, int nb, int nch, int* cand, hipStream_t st);

}  // namespace hss

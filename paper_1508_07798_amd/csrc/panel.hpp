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

// Launch gj_panel_rot_kernel for nn boxes (descriptors on the device).
template <class X>
void launch_panel_rot(const GjDesc<X>* dd, int nn, int j0, int nb, const PanelShape& s, hipStream_t st);

// Tournament pivoting for panels above the compact kernels' capacity: the width,
// the chunk of rows each local search holds (kTournChunk) and the largest number of
// candidate rows of the final search (kTournCand).
constexpr int kTournChunk = 1024;
constexpr int kTournCand = 256;
template <class X> constexpr int tourn_nb() { return std::is_same<X, cd>::value ? 8 : 16; }

// Launch the local searches (grid nch x nn) and the final search (grid nn) of one
// panel step; cand holds nn * nch * tourn_nb<X>() ints.
template <class X>
void launch_panel_tourn(const GjDesc<X>* dd, int nn, int j0, int nb, int nch, int* cand, hipStream_t st);

}  // namespace hss

// Launch table of the compact register-resident panel kernel (gj_panel_rot_kernel):
// one instantiation per scalar type, panel width, rows per thread and thread count.
// Kept in a translation unit of its own so that it compiles beside the engine.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "../../include/hss.h"
#include "common.hpp"
#include "k_gj.hpp"
#include "panel.hpp"

namespace hss {

template <class X>
bool panel_rot_config(int rows, PanelShape& s) {
  if (rows <= 128) {
    s = {16, 1, 128};
    return true;
  }
  if constexpr (sizeof(X) == 16) {
    // complex double: 16-column rows take four registers per entry, so 512-thread
    // 16-column variants would spill; 769 .. 1280 rows go to the kernel with the
    // column loop unrolled (triangular update), taller panels to 8 columns
    if (rows <= 256 * 3) {
      s = {16, (rows + 255) / 256, 256};
      return true;
    }
    if (rows <= 256 * 5) {
      s = {16, 5, 256, true};
      return true;
    }
    if (rows <= 512 * 5) {
      s = {8, std::max(3, (rows + 511) / 512), 512};
      return true;
    }
    return false;
  } else {
    if (rows <= 256 * 4) {
      s = {16, (rows + 255) / 256, 256};
      return true;
    }
    if (rows <= 512 * 4) {
      s = {16, (rows + 511) / 512, 512};
      return true;
    }
    return false;
  }
}

template <class X>
void launch_panel_rot(const GjDesc<X>* dd, int nn, int j0, int nb, const PanelShape& s, hipStream_t st) {
#define HSS_ROT(NB_, RPT_, NT_)                                                      \
  if (!s.unrolled && s.nb == NB_ && s.rpt == RPT_ && s.nt == NT_) {                  \
    gj_panel_rot_kernel<X, NB_, RPT_, NT_><<<nn, NT_, 0, st>>>(dd, j0, nb);          \
    return;                                                                          \
  }
  HSS_ROT(16, 1, 128)
  HSS_ROT(16, 1, 256) HSS_ROT(16, 2, 256) HSS_ROT(16, 3, 256)
  if constexpr (sizeof(X) != 16) {
    HSS_ROT(16, 4, 256) HSS_ROT(16, 3, 512) HSS_ROT(16, 4, 512)
  } else {
    HSS_ROT(8, 3, 512) HSS_ROT(8, 4, 512) HSS_ROT(8, 5, 512)
    if (s.unrolled && s.nb == 16 && s.rpt == 5 && s.nt == 256) {
      gj_panel_unr_kernel<X, 16, 5, 256><<<nn, 256, 0, st>>>(dd, j0, nb);
      return;
    }
  }
#undef HSS_ROT
  throw Error(HSS_EDEVICE, "no panel variant for nb " + std::to_string(s.nb) + ", rpt " + std::to_string(s.rpt) +
                               ", threads " + std::to_string(s.nt));
}

template bool panel_rot_config<float>(int, PanelShape&);
template bool panel_rot_config<double>(int, PanelShape&);
template bool panel_rot_config<cf>(int, PanelShape&);
template bool panel_rot_config<cd>(int, PanelShape&);
template void launch_panel_rot<float>(const GjDesc<float>*, int, int, int, const PanelShape&, hipStream_t);
template void launch_panel_rot<double>(const GjDesc<double>*, int, int, int, const PanelShape&, hipStream_t);
template void launch_panel_rot<cf>(const GjDesc<cf>*, int, int, int, const PanelShape&, hipStream_t);
template void launch_panel_rot<cd>(const GjDesc<cd>*, int, int, int, const PanelShape&, hipStream_t);

}  // namespace hss

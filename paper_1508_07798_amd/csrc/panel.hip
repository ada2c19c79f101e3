// Launch table of the compact register-resident panel kernel (gj_panel_rot_kernel):
// one instantiation per scalar type, panel width, rows per thread and thread count.
// Kept in a translation unit of its own so that it compiles beside the engine.
#include <hip/hip_runtime.h>

#include <string>

#include "../../include/hss.h"
#include "common.hpp"
#include "k_gj.hpp"
#include "panel.hpp"

namespace hss {

template <class X>
bool panel_rot_config(int rows, PanelShape& s) {
  // 16 columns up to RPT = 4 rows per thread (three for complex double, whose
  // 16-column rows take four registers per entry), then 8-column panels
  const int rmax16 = sizeof(X) == 16 ? 3 : 4;
  if (rows <= 128) {
    s = {16, 1, 128};
    return true;
  }
  if (rows <= 256 * rmax16) {
    s = {16, (rows + 255) / 256, 256};
    return true;
  }
  if (rows <= 512 * rmax16) {
    s = {16, (rows + 511) / 512, 512};
    return true;
  }
  if (sizeof(X) == 16 && rows <= 512 * 5) {
    s = {8, (rows + 511) / 512, 512};
    return true;
  }
  return false;
}

template <class X>
void launch_panel_rot(const GjDesc<X>* dd, int nn, int j0, int nb, const PanelShape& s, hipStream_t st) {
#define HSS_ROT(NB_, RPT_, NT_)                                                      \
  if (s.nb == NB_ && s.rpt == RPT_ && s.nt == NT_) {                                 \
    gj_panel_rot_kernel<X, NB_, RPT_, NT_><<<nn, NT_, 0, st>>>(dd, j0, nb);          \
    return;                                                                          \
  }
  HSS_ROT(16, 1, 128)
  HSS_ROT(16, 1, 256) HSS_ROT(16, 2, 256) HSS_ROT(16, 3, 256)
  HSS_ROT(16, 2, 512) HSS_ROT(16, 3, 512)
  if constexpr (sizeof(X) != 16) {
    HSS_ROT(16, 4, 256) HSS_ROT(16, 4, 512)
  } else {
    HSS_ROT(8, 4, 512) HSS_ROT(8, 5, 512)
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

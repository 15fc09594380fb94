// SAP colour sweep instantiated for F16 storage (FP32 arithmetic).
#include "dw_sap_kernel.hpp"

namespace dw {

dw_status launch_sap_colour_f16(const Geom& g, double m0, const void* v, void* z, const void* U, int colour, int nmr,
                               int z_zero, int nrhs, long long vs, long long zs, hipStream_t s, const int* rlist,
                               const void* C, double red2, const int* gate, int gs, const double* dmass) {
  return sapk::launch<float, s16, s32, s16>(g, m0, v, z, U, colour, nmr, z_zero, nrhs, vs, zs, rlist, s, C, red2, gate, gs, dmass);
}

}  // namespace dw

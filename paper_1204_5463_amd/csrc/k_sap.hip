// One colour of the Schwarz alternating procedure (paper Section 2, Alg. 2):
// dispatch on the storage precision to the instantiations in k_sap_<prec>.hip
// (the kernel itself is in dw_sap_kernel.hpp).
#include "dw_internal.hpp"

namespace dw {

#define DW_SAP_DECL(P)                                                                                           \
  dw_status launch_sap_colour_##P(const Geom& g, double m0, const void* v, void* z, const void* U, int colour,    \
                                  int nmr, int z_zero, int nrhs, long long vs, long long zs, hipStream_t s,      \
                                  const int* rlist, const void* C, double red2, const int* gate, int gs,          \
                                  const double* dmass);
DW_SAP_DECL(f64)
DW_SAP_DECL(f32)
DW_SAP_DECL(f16)
DW_SAP_DECL(bf16)
#undef DW_SAP_DECL

dw_status launch_sap_colour(const Geom& g, double m0, int prec, const void* v, void* z, const void* U, int colour,
                            int nmr, int z_zero, int nrhs, long long vs, long long zs, hipStream_t s,
                            const int* rlist, const void* C, double mr_reduction, const int* gate, int gs,
                            const double* dmass) {
  if (nrhs < 1) return DW_OK;
  const double red2 = mr_reduction * mr_reduction;
  switch (prec) {
    case DW_PREC_F64: return launch_sap_colour_f64(g, m0, v, z, U, colour, nmr, z_zero, nrhs, vs, zs, s, rlist, C, red2, gate, gs, dmass);
    case DW_PREC_F32: return launch_sap_colour_f32(g, m0, v, z, U, colour, nmr, z_zero, nrhs, vs, zs, s, rlist, C, red2, gate, gs, dmass);
    case DW_PREC_F16: return launch_sap_colour_f16(g, m0, v, z, U, colour, nmr, z_zero, nrhs, vs, zs, s, rlist, C, red2, gate, gs, dmass);
    case DW_PREC_BF16:
      return launch_sap_colour_bf16(g, m0, v, z, U, colour, nmr, z_zero, nrhs, vs, zs, s, rlist, C, red2, gate, gs, dmass);
    default: set_error("unknown precision %d", prec); return DW_EINVAL;
  }
}

}  // namespace dw

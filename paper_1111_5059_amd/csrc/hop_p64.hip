// Wilson-hop and fifth-dimension kernels for storage precision P64.  Compiled once per
// compile-time fifth-dimension extent (-DDWF_HOP_LS=0/8/12/16/32) and once for the dispatcher.
#include "hop_impl.hpp"
using namespace dwf;
#ifdef DWF_HOP_LS
DWF_HOP_LS_ONE(P64, DWF_HOP_LS)
#else
DWF_INSTANTIATE_HOP(P64)
#endif

// Wilson-hop and fifth-dimension kernels instantiated for storage precision P64.
#include "hop_impl.hpp"
using namespace dwf;
DWF_INSTANTIATE_HOP(P64)

// Wilson-hop and fifth-dimension kernels instantiated for storage precision P16.
#include "hop_impl.hpp"
using namespace dwf;
DWF_INSTANTIATE_HOP(P16)

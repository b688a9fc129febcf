// Wilson-hop and fifth-dimension kernels instantiated for storage precision PB16.
#include "hop_impl.hpp"
using namespace dwf;
DWF_INSTANTIATE_HOP(PB16)

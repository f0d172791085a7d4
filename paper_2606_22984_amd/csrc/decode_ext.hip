// Instantiations of the decode kernel (decode_impl.h) for head widths 32 and
// 64, and for models over 2^D-spin patch tokens (every head width).
#include "decode_impl.h"

namespace fvan {

FVAN_DECODE_EXT_LIST(FVAN_DECODE_INST)

}  // namespace fvan

// Launch dispatch of the KV-cached decode kernel (decode_impl.h), and its
// instantiations for single-spin models with 16-wide heads (the hot path);
// decode_ext.hip instantiates the other head widths and the token models.
#include "decode_impl.h"

namespace fvan {

int decode_tile_samples() { return 32; }

bool decode_has_tile16(const DecodeShape& sh) {
  if (sh.tokens) return sh.d_model == 128 && sh.d_head == 64;
  return sh.d_head == 16;
}

FVAN_DECODE_INST(32, 0, 16, false, 32)
FVAN_DECODE_INST(64, 0, 16, false, 32)
FVAN_DECODE_INST(128, 0, 16, false, 32)
FVAN_DECODE_INST(32, 2, 16, false, 32)
FVAN_DECODE_INST(64, 2, 16, false, 32)
FVAN_DECODE_INST(128, 2, 16, false, 32)
FVAN_DECODE_EXT_LIST(FVAN_DECODE_EXTERN)

template <int D, int MODE, int DH>
static hipError_t dispatch_tok(const DecodeShape& sh, const DecodeUnit& u0, const DecodeUnit* table, int n_units,
                               int total_tiles, int* queue, int grid, hipStream_t s) {
  if (sh.tile == 16) {
    if constexpr (DH == 16)
      if (!sh.tokens) return launch_d<D, MODE, DH, false, 16>(u0, table, n_units, total_tiles, queue, grid, s);
    if constexpr (D == 128 && DH == 64)
      if (sh.tokens) return launch_d<D, MODE, DH, true, 16>(u0, table, n_units, total_tiles, queue, grid, s);
    return hipErrorInvalidValue;
  }
  if (sh.tile != 32) return hipErrorInvalidValue;
  return sh.tokens ? launch_d<D, MODE, DH, true, 32>(u0, table, n_units, total_tiles, queue, grid, s)
                   : launch_d<D, MODE, DH, false, 32>(u0, table, n_units, total_tiles, queue, grid, s);
}

template <int D, int MODE>
static hipError_t dispatch_dh(const DecodeShape& sh, const DecodeUnit& u0, const DecodeUnit* table, int n_units,
                              int total_tiles, int* queue, int grid, hipStream_t s) {
  switch (sh.d_head) {
    case 16: return dispatch_tok<D, MODE, 16>(sh, u0, table, n_units, total_tiles, queue, grid, s);
    case 32: return dispatch_tok<D, MODE, 32>(sh, u0, table, n_units, total_tiles, queue, grid, s);
    case 64:
      if constexpr (D >= 64) return dispatch_tok<D, MODE, 64>(sh, u0, table, n_units, total_tiles, queue, grid, s);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

template <int D>
static hipError_t dispatch_mode(const DecodeShape& sh, const DecodeUnit& u0, const DecodeUnit* table, int n_units,
                                int total_tiles, int* queue, int grid, hipStream_t s) {
  switch (sh.precision) {
    case FVAN_FP32: return dispatch_dh<D, 0>(sh, u0, table, n_units, total_tiles, queue, grid, s);
    case FVAN_BF16_SPLIT: return dispatch_dh<D, 2>(sh, u0, table, n_units, total_tiles, queue, grid, s);
    default: return hipErrorInvalidValue;
  }
}

static hipError_t dispatch(const DecodeShape& sh, const DecodeUnit& u0, const DecodeUnit* table, int n_units,
                           int total_tiles, int* queue, int grid, hipStream_t s) {
  switch (sh.d_model) {
    case 32: return dispatch_mode<32>(sh, u0, table, n_units, total_tiles, queue, grid, s);
    case 64: return dispatch_mode<64>(sh, u0, table, n_units, total_tiles, queue, grid, s);
    case 128: return dispatch_mode<128>(sh, u0, table, n_units, total_tiles, queue, grid, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_decode(const DecodeShape& sh, const DecodeUnit* units_dev, int n_units, int total_tiles,
                         int* queue_counter, int grid, hipStream_t s) {
  DecodeUnit dummy{};
  return dispatch(sh, dummy, units_dev, n_units, total_tiles, queue_counter, grid, s);
}

hipError_t launch_decode_single(const DecodeShape& sh, const DecodeUnit& u, int tiles, hipStream_t s) {
  return dispatch(sh, u, nullptr, 1, tiles, nullptr, tiles, s);
}

}  // namespace fvan

// Launch parameters of the streamed advance (host and device).
#pragma once

#include <stdint.h>

namespace tvd {

// Everything one streamed launch needs besides KParams.
struct StreamParams {
  const int32_t* start;   // [n_chains + 1] chain c = blocks[start[c] .. start[c+1])
  const int32_t* blocks;  // chain members, consecutive along the streamed axis
  int n_chains;
  int n_members;          // entries of blocks
  int quads;              // tiles per block face: 1 (edge 16) or 4 (edge 32)
};

}  // namespace tvd

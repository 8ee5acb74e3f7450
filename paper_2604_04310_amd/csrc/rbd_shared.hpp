// Plain structures shared by the host runtime and the kernels.
#pragma once

#include <stdint.h>

namespace rbd {

// Threads per block of the kernels that run one instance per lane (the heavy
// kernels choose their own block size, see the launchers).
constexpr int kBlock = 256;

// Operations of a packed serving launch (equal to rbd_op's values).
constexpr int kOpFwdDyn = 0, kOpRnea = 1, kOpFwdDynVjp = 2;

// Jacobian output frames grouped by body: output slots slot[beg[i] .. beg[i+1])
// are frames of body i. Passed by value as a kernel argument.
struct JacSlots {
  int32_t n_frames;
  int16_t beg[65];
  int16_t slot[256];
};

// Descriptor table of one packed serving launch (device memory):
//   PackedHdr, int32 tile_req[n_tiles], then PackedReq[n_req] at req_offset.
// A tile is kTileLanes consecutive instances of one request.
constexpr int kTileLanes = 64;
struct PackedHdr {
  int32_t n_tiles;
  int32_t n_req;
  int32_t req_offset;  // bytes from the start of the table, 16-aligned
  int32_t pad;
};
struct PackedReq {
  const float* in[4];  // instance-major inputs (q, qd, tau | qdd, g_qdd)
  float* out[3];       // instance-major outputs
  int32_t batch;
  int32_t first_tile;
};

}  // namespace rbd

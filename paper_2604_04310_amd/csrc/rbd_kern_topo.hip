// Kernels of one compiled topology. Built once per entry of RBD_TOPOLOGIES
// and part (-DRBD_TOPO=<name> -DRBD_PART=1..8), so they compile in parallel.
// The part's function stores the address of each of its kernels in its slot
// of the topology's kernel table.
#include <hip/hip_runtime.h>

#include "rbd_kernel_ids.hpp"
#include "rbd_kernels.hpp"
#include "rbd_topologies.hpp"

#if !defined(RBD_TOPO) || !defined(RBD_PART)
#error "RBD_TOPO must name a topology and RBD_PART a part (1..8)"
#endif

#define RBD_CAT2(a, b) a##b
#define RBD_CAT(a, b) RBD_CAT2(a, b)

namespace rbd {
namespace {
#define RBD_PICK(name, fr, ...) using T_##name = Tree<fr, __VA_ARGS__>;
RBD_TOPOLOGIES(RBD_PICK)
#undef RBD_PICK
using TP = RBD_CAT(T_, RBD_TOPO);
static_assert(TP::depth_first(), "topology is not depth-first");
}  // namespace

#define RBD_NAME RBD_CAT(RBD_CAT(RBD_CAT(kernels_, RBD_TOPO), _p), RBD_PART)
void RBD_NAME(const void** fn) {
#define RBD_FILL(id, part, ...) \
  if constexpr (part == RBD_PART) fn[id] = reinterpret_cast<const void*>(&__VA_ARGS__);
  RBD_KERNELS(RBD_FILL)
#undef RBD_FILL
}

}  // namespace rbd

// Kernels of one compiled topology. Built once per entry of RBD_TOPOLOGIES
// with -DRBD_TOPO=<name>, so the topologies compile in parallel.
#include "rbd_kernels.hpp"
#include "rbd_topologies.hpp"

#ifndef RBD_TOPO
#error "RBD_TOPO must name a topology"
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

extern const LaunchTable RBD_CAT(launch_table_, RBD_TOPO);
const LaunchTable RBD_CAT(launch_table_, RBD_TOPO) = Launch<TP>::table();

}  // namespace rbd

// Kernels of one compiled topology. Built once per entry of RBD_TOPOLOGIES
// and part (-DRBD_TOPO=<name> -DRBD_PART=1..7), so they compile in parallel.
#include "rbd_kernels.hpp"
#include "rbd_topologies.hpp"

#if !defined(RBD_TOPO) || !defined(RBD_PART)
#error "RBD_TOPO must name a topology and RBD_PART a part (1..7)"
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

#define RBD_NAME RBD_CAT(RBD_CAT(RBD_CAT(launch_table_, RBD_TOPO), _p), RBD_PART)
extern const LaunchTable RBD_NAME;
const LaunchTable RBD_NAME = Launch<TP>::part<RBD_PART>();

}  // namespace rbd

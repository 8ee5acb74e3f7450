// The compiled robot topologies: name, floating base, parents (depth-first,
// parent[i] < i, -1 = world). Every kernel is instantiated ahead of time for
// each entry, one translation unit per topology. The humanoid is a floating
// pelvis with two 6-joint legs, a 3-joint waist and two 7-joint arms; the small
// trees serve closed-form checks and tests.
#pragma once

#define RBD_TOPOLOGIES(X)                                                                             \
  X(chain1, false, -1)                                                                                \
  X(chain2, false, -1, 0)                                                                             \
  X(chain3, false, -1, 0, 1)                                                                          \
  X(chain4, false, -1, 0, 1, 2)                                                                       \
  X(chain5, false, -1, 0, 1, 2, 3)                                                                    \
  X(chain6, false, -1, 0, 1, 2, 3, 4)                                                                 \
  X(chain7, false, -1, 0, 1, 2, 3, 4, 5)                                                              \
  X(chain8, false, -1, 0, 1, 2, 3, 4, 5, 6)                                                           \
  X(free1, true, -1)                                                                                  \
  X(tree12f, true, -1, 0, 1, 1, 0, 4, 5, 5, 7, 0, 9, 10)                                              \
  X(humanoid30, true, -1, 0, 1, 2, 3, 4, 5, 0, 7, 8, 9, 10, 11, 0, 13, 14, 15, 16, 17, 18, 19, 20, 21, \
    15, 23, 24, 25, 26, 27, 28)

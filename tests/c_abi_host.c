/* A plain C11 caller of librbd.so through include/rbd.h alone, with no GPU:
 * a host-only model (validation, dimensions, error reporting) and a server
 * with the host executor (submit, wait, statistics, shutdown). Prints
 * "c abi ok" and exits 0 when every check holds. */
#include <stdio.h>
#include <string.h>

#include "rbd.h"

#define CHECK(cond)                                                      \
  do {                                                                   \
    if (!(cond)) {                                                       \
      fprintf(stderr, "check failed at line %d: %s (last error: %s)\n", \
              __LINE__, #cond, rbd_last_error());                        \
      return 1;                                                          \
    }                                                                    \
  } while (0)

int main(void) {
  /* a three-link arm: revolute joints about z, links 0.3 m along x */
  const int32_t parent[3] = {-1, 0, 1};
  const int32_t joint[3] = {RBD_JOINT_REVOLUTE, RBD_JOINT_REVOLUTE, RBD_JOINT_REVOLUTE};
  double axis[9], origin[36], mass[3], com[9], inertia[18];
  for (int i = 0; i < 3; ++i) {
    const double o[12] = {1, 0, 0, 0, 1, 0, 0, 0, 1, i ? 0.3 : 0.0, 0, 0};
    memcpy(origin + 12 * i, o, sizeof o);
    axis[3 * i] = 0, axis[3 * i + 1] = 0, axis[3 * i + 2] = 1;
    mass[i] = 1.0 + i;
    com[3 * i] = 0.15, com[3 * i + 1] = 0, com[3 * i + 2] = 0;
    const double in[6] = {0.01, 0.02, 0.02, 0, 0, 0};
    memcpy(inertia + 6 * i, in, sizeof in);
  }
  rbd_tree_desc d = {3, parent, joint, axis, origin, mass, com, inertia, {0.0, 0.0, -9.81}};

  rbd_model* m = NULL;
  CHECK(rbd_model_create(&d, -1, &m) == RBD_OK && m != NULL);
  int nq = 0, nv = 0, nb = 0;
  CHECK(rbd_model_dims(m, &nq, &nv, &nb) == RBD_OK && nq == 3 && nv == 3 && nb == 3);
  CHECK(rbd_model_topology(m) != NULL);

  /* a host-only model has no kernels: compute calls report it */
  float x[3] = {0, 0, 0}, y[3];
  CHECK(rbd_fwd_dyn(m, 1, 1, x, x, x, NULL, y, NULL) == RBD_E_NODEVICE);

  /* an invalid tree is rejected with a message */
  const int32_t bad_parent[3] = {-1, 1, 1};
  rbd_tree_desc bad = d;
  bad.parent = bad_parent;
  rbd_model* mb = NULL;
  CHECK(rbd_model_create(&bad, -1, &mb) == RBD_E_INVAL && mb == NULL);
  CHECK(strlen(rbd_last_error()) > 0);
  CHECK(strcmp(rbd_status_str(RBD_E_INVAL), rbd_status_str(RBD_OK)) != 0);

  /* the server's scheduler with the host executor */
  rbd_server_config cfg;
  memset(&cfg, 0, sizeof cfg);
  cfg.arena_bytes = 1 << 20;
  cfg.n_streams = 2;
  cfg.max_batch_requests = 16;
  cfg.executor = RBD_EXEC_HOST;
  rbd_server* s = NULL;
  CHECK(rbd_server_create(&cfg, &s) == RBD_OK && s != NULL);
  enum { B = 5 };
  float q[B][3], qd[B][3], tau[B][3], qdd[B][3];
  for (int i = 0; i < B; ++i)
    for (int c = 0; c < 3; ++c) {
      q[i][c] = (float)(10 * i + c);
      qd[i][c] = -q[i][c];
      tau[i][c] = 0.5f * q[i][c];
      qdd[i][c] = -1.0f;
    }
  const float* in[3] = {&q[0][0], &qd[0][0], &tau[0][0]};
  float* out[1] = {&qdd[0][0]};
  uint64_t ticket = 0;
  CHECK(rbd_server_submit(s, m, RBD_OP_FWD_DYN, B, in, out, &ticket) == RBD_OK);
  rbd_status req = RBD_E_LAUNCH;
  CHECK(rbd_server_wait(s, ticket, 10.0, &req) == RBD_OK && req == RBD_OK);
  /* the host executor's stand-in: output 0 repeats input 0 */
  for (int i = 0; i < B; ++i)
    for (int c = 0; c < 3; ++c) CHECK(qdd[i][c] == q[i][c]);
  rbd_server_stats st;
  CHECK(rbd_server_get_stats(s, &st) == RBD_OK && st.requests == 1 && st.instances == B);
  CHECK(rbd_server_submit(s, m, 99, B, in, out, &ticket) == RBD_E_INVAL);
  CHECK(rbd_server_destroy(s) == RBD_OK);
  CHECK(rbd_model_destroy(m) == RBD_OK);
  printf("c abi ok\n");
  return 0;
}

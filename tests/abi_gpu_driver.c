/* The C ABI used from plain C on the GPU (no Python, no torch): device buffers from hipMalloc,
 * one eager rgp_correct, then a captured plan (rgp_correct_plan) replayed twice on a stream of its
 * own.  Reads two FP32 volumes (raw, caller layout m0 x m1 x m2) from files, writes the eager
 * field (FP32, staggered along pe) and prints whether every replay equals the eager result byte
 * for byte.
 *
 *   abi_gpu_driver I_plus.f32 I_minus.f32 m0 m1 m2 pe levels gn_iters pcg_iters b_out.f32
 *
 * Exit status 0 when every call returned RGP_OK and the replays matched. */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../include/rgp.h"

#define HIP_OK(call)                                                              \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess) {                                                       \
      fprintf(stderr, "%s failed: %s\n", #call, hipGetErrorString(e_));           \
      return 2;                                                                   \
    }                                                                             \
  } while (0)
#define RGP_OK_(call)                                                             \
  do {                                                                            \
    rgp_status s_ = (call);                                                       \
    if (s_ != RGP_OK) {                                                           \
      fprintf(stderr, "%s failed: %s\n", #call, rgp_status_string(s_));           \
      return 3;                                                                   \
    }                                                                             \
  } while (0)

static int read_file(const char* path, void* dst, size_t bytes) {
  FILE* f = fopen(path, "rb");
  if (!f) return 1;
  const size_t got = fread(dst, 1, bytes, f);
  fclose(f);
  return got != bytes;
}

int main(int argc, char** argv) {
  if (argc != 11) {
    fprintf(stderr, "usage: %s I_plus I_minus m0 m1 m2 pe levels gn_iters pcg_iters b_out\n",
            argv[0]);
    return 1;
  }
  rgp_grid g;
  memset(&g, 0, sizeof g);
  for (int d = 0; d < 3; ++d) {
    g.m[d] = atoll(argv[3 + d]);
    g.h[d] = 1.0;
  }
  g.pe = atoi(argv[6]);
  rgp_solver_opts o;
  rgp_default_opts(&o);
  o.levels = atoi(argv[7]);
  o.gn_iters = atoi(argv[8]);
  o.pcg_iters = atoi(argv[9]);
  o.pcg_rtol = 0.0;

  const size_t ncell = (size_t)(g.m[0] * g.m[1] * g.m[2]);
  const size_t nnode = ncell / (size_t)g.m[g.pe] * (size_t)(g.m[g.pe] + 1);
  const size_t ci = ncell * sizeof(float), cb = nnode * sizeof(float);
  float* host = (float*)malloc(ci > cb ? ci : cb);
  float* host2 = (float*)malloc(cb);
  if (!host || !host2) return 1;

  void *Ip, *Im, *b, *b2, *ws;
  size_t ws_bytes = 0;
  RGP_OK_(rgp_workspace_size(RGP_OP_CORRECT, &g, RGP_F32, &o, &ws_bytes));
  HIP_OK(hipMalloc(&Ip, ci));
  HIP_OK(hipMalloc(&Im, ci));
  HIP_OK(hipMalloc(&b, cb));
  HIP_OK(hipMalloc(&b2, cb));
  HIP_OK(hipMalloc(&ws, ws_bytes));
  HIP_OK(hipMemset(ws, 0, ws_bytes));
  if (read_file(argv[1], host, ci)) return 1;
  HIP_OK(hipMemcpy(Ip, host, ci, hipMemcpyHostToDevice));
  if (read_file(argv[2], host, ci)) return 1;
  HIP_OK(hipMemcpy(Im, host, ci, hipMemcpyHostToDevice));
  hipStream_t s;
  HIP_OK(hipStreamCreate(&s));

  /* eager correction */
  RGP_OK_(rgp_correct(&g, RGP_F32, Ip, Im, RGP_F32, &o, NULL, b, NULL, NULL, NULL, ws, ws_bytes,
                      (void*)s));
  HIP_OK(hipStreamSynchronize(s));
  HIP_OK(hipMemcpy(host, b, cb, hipMemcpyDeviceToHost));

  /* the same correction captured once and replayed twice into another output buffer */
  rgp_plan plan = NULL;
  RGP_OK_(rgp_correct_plan(&g, RGP_F32, Ip, Im, RGP_F32, &o, NULL, b2, NULL, NULL, NULL, ws,
                           ws_bytes, (void*)s, &plan));
  int same = 1;
  for (int r = 0; r < 2; ++r) {
    HIP_OK(hipMemset(b2, 0xff, cb));
    RGP_OK_(rgp_plan_launch(plan, (void*)s));
    HIP_OK(hipStreamSynchronize(s));
    HIP_OK(hipMemcpy(host2, b2, cb, hipMemcpyDeviceToHost));
    same = same && memcmp(host, host2, cb) == 0;
  }
  RGP_OK_(rgp_plan_destroy(plan));

  FILE* f = fopen(argv[10], "wb");
  if (!f || fwrite(host, 1, cb, f) != cb) return 1;
  fclose(f);
  printf("abi_gpu_driver: %lld x %lld x %lld pe %d, %zu field nodes, replays equal eager: %s\n",
         (long long)g.m[0], (long long)g.m[1], (long long)g.m[2], g.pe, nnode,
         same ? "yes" : "no");
  HIP_OK(hipStreamDestroy(s));
  hipFree(Ip);
  hipFree(Im);
  hipFree(b);
  hipFree(b2);
  hipFree(ws);
  free(host);
  free(host2);
  return same ? 0 : 4;
}

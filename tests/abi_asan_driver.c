/* Host-side checks of the C ABI under AddressSanitizer: every entry point's argument validation,
 * the workspace size computations (including the batched plan's dry recording and launch-table
 * merge) and the status strings, all of which run on the host without touching a GPU.  Exits 0
 * when every returned status is the expected one; AddressSanitizer aborts on a memory error. */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "rgp.h"

static int failures = 0;
#define EXPECT(call, want)                                                       \
  do {                                                                           \
    int got_ = (int)(call);                                                      \
    if (got_ != (want)) {                                                        \
      fprintf(stderr, "%s:%d: %s returned %d, expected %d\n", __FILE__, __LINE__, \
              #call, got_, (int)(want));                                         \
      ++failures;                                                                \
    }                                                                            \
  } while (0)

static rgp_grid grid(int64_t m0, int64_t m1, int64_t m2, int pe) {
  rgp_grid g;
  memset(&g, 0, sizeof g);
  g.m[0] = m0;
  g.m[1] = m1;
  g.m[2] = m2;
  g.pe = pe;
  g.h[0] = g.h[1] = g.h[2] = 1.0;
  return g;
}

int main(void) {
  for (int s = -9; s <= 1; ++s) {
    const char* t = rgp_status_string((rgp_status)s);
    if (!t || !t[0]) ++failures;
  }
  rgp_solver_opts o;
  rgp_default_opts(&o);
  size_t n = 0;
  rgp_grid g = grid(144, 168, 111, 1);
  for (int op = 0; op < 6; ++op) {
    o.levels = 3;
    for (int solver = 0; solver < 3; ++solver) {
      o.solver = solver;
      EXPECT(rgp_workspace_size((rgp_op)op, &g, RGP_F32, &o, &n), RGP_OK);
      if (n == 0 || n % 256) ++failures;
    }
  }
  o.solver = RGP_SOLVER_LBFGS;
  o.lbfgs_memory = 40;
  EXPECT(rgp_workspace_size(RGP_OP_CORRECT, &g, RGP_F32, &o, &n), RGP_EINVAL);
  rgp_default_opts(&o);
  o.batch_march = 65;
  EXPECT(rgp_workspace_size(RGP_OP_CORRECT, &g, RGP_F32, &o, &n), RGP_EINVAL);
  o.batch_march = -1;
  EXPECT(rgp_workspace_size(RGP_OP_CORRECT, &g, RGP_F32, &o, &n), RGP_EINVAL);
  o.batch_march = 64;
  EXPECT(rgp_workspace_size(RGP_OP_CORRECT, &g, RGP_F32, &o, &n), RGP_OK);
  rgp_default_opts(&o);
  rgp_grid bad = grid(144, 1, 111, 1);
  EXPECT(rgp_workspace_size(RGP_OP_LOSS_GRAD, &bad, RGP_F32, NULL, &n), RGP_ESHAPE);
  bad = grid(16, 16, 513, 1);
  EXPECT(rgp_workspace_size(RGP_OP_LOSS_GRAD, &bad, RGP_F32, NULL, &n), RGP_ESHAPE);
  EXPECT(rgp_workspace_size(RGP_OP_LOSS_GRAD, &g, RGP_BF16, NULL, &n), RGP_EDTYPE);
  EXPECT(rgp_workspace_size(RGP_OP_LOSS_GRAD, NULL, RGP_F32, NULL, &n), RGP_EINVAL);

  /* the batched plan's workspace: a dry recording of every pair and the merge of the launch
   * sequences into shared launches (host containers only) */
  rgp_grid gs[4] = {grid(40, 48, 36, 1), grid(45, 30, 26, 0), grid(33, 41, 29, 1),
                    grid(28, 36, 44, 0)};
  for (int solver = 0; solver < 3; ++solver) {
    rgp_default_opts(&o);
    o.levels = 2;
    o.gn_iters = 3;
    o.pcg_iters = 5;
    o.solver = solver;
    EXPECT(rgp_batch_workspace_size(4, gs, RGP_F32, &o, &n), RGP_OK);
    if (n == 0) ++failures;
  }
  EXPECT(rgp_batch_workspace_size(0, gs, RGP_F32, &o, &n), RGP_EINVAL);

  /* argument errors of the enqueueing entry points: returned before any device work */
  void* fake = (void*)0x1000;
  g = grid(8, 9, 10, 1);
  EXPECT(rgp_loss_grad(&g, RGP_F32, fake, fake, RGP_F32, fake, 300.0, 1e-4, fake, NULL, NULL,
                       NULL, NULL, 0, NULL), RGP_EWORKSPACE);
  EXPECT(rgp_loss_grad(&g, RGP_F32, fake, fake, RGP_F32, NULL, 300.0, 1e-4, fake, NULL, NULL,
                       NULL, fake, 1 << 30, NULL), RGP_EINVAL);
  EXPECT(rgp_loss_grad_noalloc(&g, RGP_F64, fake, fake, RGP_F32, fake, 300.0, 1e-4, fake, NULL,
                               NULL, NULL, NULL), RGP_EDTYPE);
  EXPECT(rgp_gn_hvp(&g, RGP_F32, NULL, fake, 300.0, fake, fake, NULL, fake, 1 << 30, NULL),
         RGP_EINVAL);
  EXPECT(rgp_pcg_solve(&g, RGP_F32, fake, fake, 300.0, fake, fake, 0, 0.1, NULL, NULL, fake,
                       1 << 30, NULL), RGP_EINVAL);
  EXPECT(rgp_ot_init(&g, RGP_BF16, fake, fake, RGP_BF16, fake, 1e-3, 1, NULL, fake, 1 << 30,
                     NULL), RGP_EDTYPE);
  EXPECT(rgp_correct_lsq(&g, RGP_F32, fake, fake, RGP_F32, fake, 0, 1e-6, fake, NULL, NULL),
         RGP_EINVAL);
  rgp_grid glong = grid(4000, 2, 2, 0);
  EXPECT(rgp_correct_lsq(&glong, RGP_F32, fake, fake, RGP_F32, fake, 10, 1e-6, fake, NULL, NULL),
         RGP_ESHAPE);
  rgp_default_opts(&o);
  o.use_b_init = 1;
  EXPECT(rgp_correct(&g, RGP_F32, fake, fake, RGP_F32, &o, NULL, fake, NULL, NULL, NULL, fake,
                     1 << 30, NULL), RGP_EINVAL);
  rgp_default_opts(&o);
  o.solver = RGP_SOLVER_ADMM;
  o.alpha = 0.0;
  EXPECT(rgp_correct(&g, RGP_F32, fake, fake, RGP_F32, &o, NULL, fake, NULL, NULL, NULL, fake,
                     1 << 30, NULL), RGP_EINVAL);
  rgp_default_opts(&o);
  o.solver = RGP_SOLVER_ADMM;
  rgp_grid gpe = grid(600, 4, 4, 0);   /* more than 512 field nodes along PE */
  EXPECT(rgp_correct(&gpe, RGP_F32, fake, fake, RGP_F32, &o, NULL, fake, NULL, NULL, NULL, fake,
                     1 << 30, NULL), RGP_ESHAPE);
  rgp_default_opts(&o);
  EXPECT(rgp_correct(&g, RGP_F32, fake, fake, RGP_F32, &o, NULL, fake, NULL, NULL, NULL,
                     (void*)0x1004, 1 << 30, NULL), RGP_EWORKSPACE);
  EXPECT(rgp_blur_field(&g, RGP_F32, fake, fake, NULL), RGP_EINVAL);
  /* pyramid transfers of images: distinct buffers, field-type results, extents >= 1 */
  EXPECT(rgp_restrict_image(&g, RGP_F32, fake, RGP_F32, fake, NULL), RGP_EINVAL);
  EXPECT(rgp_restrict_image(&g, RGP_F32, fake, RGP_BF16, (void*)0x2000, NULL), RGP_EDTYPE);
  EXPECT(rgp_restrict_image(NULL, RGP_F32, fake, RGP_F32, (void*)0x2000, NULL), RGP_EINVAL);
  rgp_grid g0 = grid(0, 4, 4, 1);
  EXPECT(rgp_restrict_image(&g0, RGP_F32, fake, RGP_F32, (void*)0x2000, NULL), RGP_ESHAPE);
  EXPECT(rgp_restrict_image_adjoint(&g, RGP_BF16, fake, (void*)0x2000, 0, NULL), RGP_EDTYPE);
  EXPECT(rgp_restrict_image_adjoint(&g, RGP_F64, fake, fake, 1, NULL), RGP_EINVAL);
  EXPECT(rgp_restrict_image_adjoint(&g, RGP_F64, NULL, fake, 0, NULL), RGP_EINVAL);
  EXPECT(rgp_plan_launch(NULL, NULL), RGP_EINVAL);
  if (failures) {
    fprintf(stderr, "%d unexpected status codes\n", failures);
    return 1;
  }
  printf("abi asan driver: all checks passed\n");
  return 0;
}

/* Host-side checks of libofv under AddressSanitizer: every entry point on a
 * validation-only handle (device -1), which validates its arguments and
 * plans the call exactly as on a device but launches nothing.  Built and run
 * by tests/test_asan_host.py; exits 0 when every status is the expected one
 * (memory errors abort the process through the sanitizer). */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "ofv.h"
#include "ofv_stages.h"

static int failures = 0;

static void expect(const char* what, ofv_status got, ofv_status want) {
  if (got != want) {
    fprintf(stderr, "%s: status %d, expected %d\n", what, (int)got, (int)want);
    ++failures;
  }
}

static ofv_image img(uintptr_t addr, int w, int h, int type, int bits) {
  ofv_image i;
  i.data = (const void*)addr;
  i.width = w;
  i.height = h;
  i.pitch = w;
  i.type = type;
  i.bit_depth = bits;
  return i;
}

/* deterministic text for the tuning-table parser */
static uint32_t rng = 12345u;
static uint32_t next_rand(void) {
  rng = rng * 1664525u + 1013904223u;
  return rng >> 8;
}

int main(void) {
  ofv_handle h = NULL;
  expect("create", ofv_create(&h, -1, 256, 128, 4, NULL), OFV_OK);
  if (!h) return 1;
  ofv_handle bad = NULL;
  expect("create 0x0", ofv_create(&bad, -1, 0, 16, 1, NULL), OFV_ERR_INVALID_ARG);
  (void)ofv_last_error(NULL);
  size_t bytes = 0;
  expect("workspace bytes", ofv_workspace_bytes(h, &bytes), OFV_OK);

  ofv_params p;
  ofv_default_params(&p);
  ofv_image f0 = img(0x100000, 64, 32, OFV_PIX_U8, 8), f1 = img(0x200000, 64, 32, OFV_PIX_U8, 8);
  float* out = (float*)(uintptr_t)0x90000000u;
  expect("compute", ofv_compute_flow(h, &f0, &f1, &p, out), OFV_ERR_UNSUPPORTED);
  expect("compute null", ofv_compute_flow(h, NULL, &f1, &p, out), OFV_ERR_INVALID_ARG);
  ofv_params q = p;
  q.kernel_radius = 0;
  expect("compute kr 0", ofv_compute_flow(h, &f0, &f1, &q, out), OFV_ERR_INVALID_ARG);
  q = p;
  q.flags = 1u << 20;
  expect("compute flags", ofv_compute_flow(h, &f0, &f1, &q, out), OFV_ERR_INVALID_ARG);
  ofv_image big = img(0x100000, 512, 32, OFV_PIX_U8, 8);
  expect("compute too big", ofv_compute_flow(h, &big, &big, &p, out), OFV_ERR_CAPACITY);
  expect("compute overlap", ofv_compute_flow(h, &f0, &f1, &p, (float*)(uintptr_t)0x100010), OFV_ERR_INVALID_ARG);
  expect("compute ex", ofv_compute_flow_ex(h, &f0, &f1, &p, out, out), OFV_ERR_UNSUPPORTED);

  /* batches of uneven sizes, and one too many */
  ofv_image b0[5], b1[5];
  float* bo[5];
  const float* bi[5];
  for (int j = 0; j < 5; ++j) {
    b0[j] = img(0x1000000 + 0x100000 * (uintptr_t)j, 64 + 16 * j, 32 + 8 * j, OFV_PIX_U16, 12);
    b1[j] = img(0x2000000 + 0x100000 * (uintptr_t)j, 64 + 16 * j, 32 + 8 * j, OFV_PIX_U16, 12);
    bo[j] = (float*)(uintptr_t)(0x80000000u + 0x1000000u * (uintptr_t)j);
    bi[j] = j % 2 ? NULL : (const float*)(uintptr_t)(0x40000000u + 0x1000000u * (uintptr_t)j);
  }
  expect("batch", ofv_compute_flow_batch(h, 4, b0, b1, &p, bi, bo), OFV_ERR_UNSUPPORTED);
  expect("batch 5", ofv_compute_flow_batch(h, 5, b0, b1, &p, bi, bo), OFV_ERR_CAPACITY);
  q = p;
  q.flags = OFV_FLAG_SAVE_ITERATES;
  expect("batch saving, no reservation", ofv_compute_flow_batch(h, 4, b0, b1, &q, bi, bo), OFV_ERR_CAPACITY);
  expect("static saving", ofv_compute_flow_static(&f0, &f1, &q, out, NULL), OFV_ERR_UNSUPPORTED);

  /* backward */
  expect("backward workspace", ofv_backward_workspace_bytes(h, 3, 3, 4, OFV_BACKWARD_STORE_ALL, &bytes), OFV_OK);
  expect("reserve", ofv_reserve_backward_ex(h, 3, 3, 2, 0), OFV_ERR_UNSUPPORTED);
  const float* gf[4] = {(const float*)(uintptr_t)0xA0000000u, (const float*)(uintptr_t)0xA1000000u,
                        (const float*)(uintptr_t)0xA2000000u, (const float*)(uintptr_t)0xA3000000u};
  float* g0[4] = {(float*)(uintptr_t)0xB0000000u, NULL, (float*)(uintptr_t)0xB2000000u, NULL};
  expect("backward batch", ofv_compute_flow_backward_batch(h, 4, b0, b1, &p, bi, gf, g0, NULL, NULL),
         OFV_ERR_CAPACITY);
  float* g0o[4] = {(float*)(uintptr_t)0x2000000u, NULL, NULL, NULL};
  expect("backward batch overlap", ofv_compute_flow_backward_batch(h, 4, b0, b1, &p, bi, gf, g0o, NULL, NULL),
         OFV_ERR_INVALID_ARG);
  expect("backward", ofv_compute_flow_backward(h, &f0, &f1, &p, NULL, gf[0], g0[0], NULL, NULL), OFV_ERR_CAPACITY);

  /* decompositions and the tuning table: export, re-import, and malformed text */
  expect("variant", ofv_set_gn_variant(h, OFV_GN_TILE_64x16, 0), OFV_OK);
  expect("variant bad", ofv_set_gn_variant(h, 99, 0), OFV_ERR_INVALID_ARG);
  expect("import", ofv_tuning_import(h, "4 0 1 1024 1024 1 2 16\n10 0 1 5120 4096 1 11 0\n"), OFV_OK);
  size_t need = 0;
  expect("export size", ofv_tuning_export(h, NULL, 0, &need), OFV_OK);
  char* buf = (char*)malloc(need);
  expect("export", ofv_tuning_export(h, buf, need, &need), OFV_OK);
  expect("export short", ofv_tuning_export(h, buf, need / 2, &need), OFV_ERR_CAPACITY);
  expect("reimport", ofv_tuning_import(h, buf), OFV_OK);
  free(buf);
  const char alphabet[] = "0123456789 -\n\tx";
  for (int t = 0; t < 2000; ++t) {
    char text[96];
    const int n = (int)(next_rand() % 95);
    for (int k = 0; k < n; ++k) text[k] = alphabet[next_rand() % (sizeof(alphabet) - 1)];
    text[n] = 0;
    (void)ofv_tuning_import(h, text);
  }
  expect("autotune", ofv_autotune(h, &f0, &f1, &p, out, 1), OFV_ERR_UNSUPPORTED);
  expect("autotune batch", ofv_autotune_batch(h, 4, b0, b1, &p, bo, 1), OFV_ERR_UNSUPPORTED);

  /* streaming, derived quantities, stages */
  int produced = 0;
  expect("push", ofv_stream_push(h, &f0, &p, NULL, out, &produced), OFV_ERR_UNSUPPORTED);
  expect("reset", ofv_stream_reset(h), OFV_OK);
  ofv_derived_params dp;
  ofv_default_derived_params(&dp);
  expect("derived", ofv_derived(h, out, 64, 32, 64, NULL, 0, &dp, (float*)(uintptr_t)0xC0000000u, 64, NULL, 0,
                                NULL, NULL), OFV_ERR_UNSUPPORTED);
  dp.dt = 0.0f;
  expect("derived dt 0", ofv_derived(h, out, 64, 32, 64, NULL, 0, &dp, NULL, 0, NULL, 0, NULL, NULL),
         OFV_ERR_INVALID_ARG);
  expect("stage normalize", ofv_stage_normalize(h, &f0, 2, 1e-4f, OFV_STORE_F32, out, 64), OFV_ERR_UNSUPPORTED);
  void* outs[3] = {(void*)(uintptr_t)0xD0000000u, (void*)(uintptr_t)0xD1000000u, (void*)(uintptr_t)0xD2000000u};
  int64_t pitches[3] = {32, 16, 8};
  expect("stage pyramid", ofv_stage_pyramid(h, OFV_STORE_F32, (const void*)(uintptr_t)0xE0000000u, 64, 32, 64, 3,
                                            outs, pitches), OFV_ERR_UNSUPPORTED);
  expect("stage pyramid 4", ofv_stage_pyramid(h, OFV_STORE_F32, (const void*)(uintptr_t)0xE0000000u, 64, 32, 64, 4,
                                              outs, pitches), OFV_ERR_INVALID_ARG);
  expect("stage gn", ofv_stage_gn_iteration(h, OFV_STORE_F32, (const void*)(uintptr_t)0xE0000000u,
                                            (const void*)(uintptr_t)0xE1000000u, 64, 32, 64, OFV_FLOW_IN_ZERO, NULL,
                                            0, 0, 0, out, 64, 4, 1e-3f, 1e-9f), OFV_ERR_UNSUPPORTED);
  for (int s = -6; s <= 1; ++s) (void)ofv_status_string((ofv_status)s);
  (void)ofv_last_error(h);
  expect("destroy", ofv_destroy(h), OFV_OK);
  expect("destroy null", ofv_destroy(NULL), OFV_OK);
  if (failures) fprintf(stderr, "%d unexpected statuses\n", failures);
  else printf("asan driver: all statuses as expected\n");
  return failures ? 2 : 0;
}

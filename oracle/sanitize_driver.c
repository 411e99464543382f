/* Test infrastructure: a stand-alone driver of the oracle, built with
 * AddressSanitizer and UndefinedBehaviorSanitizer by the CPU tests.  It reads
 * a scene file, runs a schedule of render iterations and updates (the first
 * classic RR, the rest MARS), and writes every iteration's per-sample
 * radiance, so that a test can compare it with the oracle library run on the
 * same scene.
 *
 * Scene file (little endian): int32 ntri, nmat, ncam, width, height; float32
 * V[ntri][9]; uint32 tri_mat[ntri]; float32 mats[nmat][8]; float32 cam[ncam].
 * Usage: sanitize_driver scene mode max_depth lp_classes iterations spp
 *        stat_clamp out
 */
#include <stdio.h>
#include <stdlib.h>

#include "oracle.h"

static void* read_n(FILE* f, size_t bytes) {
  void* p = malloc(bytes ? bytes : 1);
  if (!p || fread(p, 1, bytes, f) != bytes) {
    fprintf(stderr, "scene file truncated\n");
    exit(2);
  }
  return p;
}

int main(int argc, char** argv) {
  if (argc != 9) {
    fprintf(stderr, "usage: %s scene mode max_depth lp_classes iterations spp stat_clamp out\n",
            argv[0]);
    return 2;
  }
  FILE* f = fopen(argv[1], "rb");
  if (!f) return 2;
  int32_t hdr[5];
  if (fread(hdr, sizeof(int32_t), 5, f) != 5) return 2;
  const int32_t ntri = hdr[0], nmat = hdr[1], ncam = hdr[2], W = hdr[3], H = hdr[4];
  float* V = (float*)read_n(f, sizeof(float) * 9 * (size_t)ntri);
  uint32_t* tm = (uint32_t*)read_n(f, sizeof(uint32_t) * (size_t)ntri);
  float* mats = (float*)read_n(f, sizeof(float) * 8 * (size_t)nmat);
  float* cam = (float*)read_n(f, sizeof(float) * (size_t)ncam);
  fclose(f);

  orc_config cfg = {0};
  cfg.mode = atoi(argv[2]);
  cfg.max_depth = atoi(argv[3]);
  cfg.max_cells = 65536;
  cfg.max_tree_depth = 8;
  cfg.split_visits = 32;
  cfg.nee_enabled = 1;
  cfg.seed = 1;
  cfg.lp_classes = atoi(argv[4]);
  const int iters = atoi(argv[5]), spp = atoi(argv[6]);
  const float stat_clamp = (float)atof(argv[7]);
  oracle* o = orc_create(V, tm, ntri, mats, nmat, cam, W, H, &cfg);
  if (!o) {
    fprintf(stderr, "invalid scene\n");
    return 3;
  }
  FILE* out = fopen(argv[8], "wb");
  if (!out) return 2;
  const size_t n = (size_t)W * H * spp * 3;
  float* L = (float*)malloc(sizeof(float) * n);
  for (int it = 0; it < iters; ++it) {
    /* the oracle library's default parameters */
    orc_iter_params p = {0};
    p.iteration = it;
    p.spp = spp;
    p.alloc = it == 0 ? ORC_ALLOC_CLASSIC : ORC_ALLOC_MARS;
    p.budget_aware = 1;
    p.rr_start = 5;
    p.clamp_lo = 0.05f;
    p.clamp_hi = 20.0f;
    p.stat_clamp = stat_clamp;
    p.lp_stride = 7919;
    orc_iter_stats st;
    orc_update_stats us;
    if (orc_render_iteration(o, &p, &st) != 0) return 4;
    orc_read_sample_radiance(o, L);
    if (fwrite(L, sizeof(float), n, out) != n) return 2;
    if (orc_update(o, &p, &us) != 0) return 4;
  }
  fclose(out);
  free(L);
  orc_destroy(o);
  free(V);
  free(tm);
  free(mats);
  free(cam);
  return 0;
}

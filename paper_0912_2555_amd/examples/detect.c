/*
 * Using libmapcheck from C, with no Python: upload an edge list, build the
 * pull CSR on the device, run the MAP outer loop (map_detect) and ask for a
 * counterexample of the cycle it reports (map_lasso).
 *
 * Two graphs, with the results their construction fixes:
 *   - the worked example 1->2, 2->3, 3->1, 3->4, 4->5 with accepting {2, 4, 5}:
 *     the maximal accepting successors are 5 5 5 5 0, then 4 4 4 0 0, then
 *     2 2 2 0 0, where vertex 2 is its own: found, witness 2, K = 3; from
 *     vertex 1 the lasso is 1->2 then 2->3->1->2;
 *   - a ring 1->2->...->600->1 entered by a tail 601->602->...->1000->1, every
 *     seventh id accepting: ring vertices reach only the ring, whose largest
 *     accepting id is 595, so 595 is its own maximal accepting successor in
 *     the first iteration (K = 1, witness 595); from 601 the shortest path to
 *     595 runs down the tail and around the ring (399 + 1 + 594 edges) and the
 *     cycle is the whole ring (600 edges).
 * Prints one line per graph and exits with 0 when every value matches.
 *
 * Build (next to libmapcheck.so):
 *   gcc -std=c11 -D__HIP_PLATFORM_AMD__ -I/opt/rocm/include -I include \
 *       paper_0912_2555_amd/examples/detect.c -L paper_0912_2555_amd -lmapcheck \
 *       -L/opt/rocm/lib -lamdhip64 -Wl,-rpath,'$ORIGIN/..' -Wl,-rpath,/opt/rocm/lib \
 *       -o paper_0912_2555_amd/examples/detect
 */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "mapcheck.h"

#define CHECK_HIP(x)                                                        \
  do {                                                                      \
    hipError_t e_ = (x);                                                    \
    if (e_ != hipSuccess) {                                                 \
      fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));               \
      exit(2);                                                              \
    }                                                                       \
  } while (0)

#define CHECK_MAP(x)                                                        \
  do {                                                                      \
    int r_ = (x);                                                           \
    if (r_ != MAP_OK) {                                                     \
      fprintf(stderr, "%s: %s\n", #x, map_strerror(r_));                    \
      exit(2);                                                              \
    }                                                                       \
  } while (0)

typedef struct {
  int32_t found, witness, iterations, stem, cycle;
} outcome;

/* Detect on one graph (1-based edge list src[i] -> dst[i]) and, if a cycle is
 * found, build the lasso from vertex `init`. */
static outcome run(int32_t n, int64_t m, const int32_t* src, const int32_t* dst, const uint8_t* acc,
                   int32_t init) {
  int32_t *d_src, *d_dst, *row_ptr, *col, *status, *path;
  uint8_t* d_acc;
  map_result* d_res;
  map_lasso_result* d_lasso;
  void* ws;
  const size_t ws_bytes = map_workspace_bytes(n, m, 0);
  const int32_t cap = 2 * n + 1;
  CHECK_HIP(hipMalloc((void**)&d_src, (size_t)m * 4));
  CHECK_HIP(hipMalloc((void**)&d_dst, (size_t)m * 4));
  CHECK_HIP(hipMalloc((void**)&d_acc, (size_t)n));
  CHECK_HIP(hipMalloc((void**)&row_ptr, ((size_t)n + 1) * 4));
  CHECK_HIP(hipMalloc((void**)&col, (size_t)m * 4));
  CHECK_HIP(hipMalloc((void**)&status, 4));
  CHECK_HIP(hipMalloc((void**)&d_res, sizeof(map_result)));
  CHECK_HIP(hipMalloc((void**)&d_lasso, sizeof(map_lasso_result)));
  CHECK_HIP(hipMalloc((void**)&path, (size_t)cap * 4));
  CHECK_HIP(hipMalloc(&ws, ws_bytes));
  CHECK_HIP(hipMemcpy(d_src, src, (size_t)m * 4, hipMemcpyHostToDevice));
  CHECK_HIP(hipMemcpy(d_dst, dst, (size_t)m * 4, hipMemcpyHostToDevice));
  CHECK_HIP(hipMemcpy(d_acc, acc, (size_t)n, hipMemcpyHostToDevice));

  CHECK_MAP(map_build_csr(n, m, d_src, d_dst, row_ptr, col, NULL, NULL, status, ws, ws_bytes, NULL));
  CHECK_MAP(map_detect(n, row_ptr, col, NULL, NULL, d_acc, d_res, NULL, 0, NULL, 0, 0, ws, ws_bytes, NULL));
  map_result r;
  CHECK_HIP(hipMemcpy(&r, d_res, sizeof(r), hipMemcpyDeviceToHost));  /* synchronizes the stream */
  int32_t build_status = 0;
  CHECK_HIP(hipMemcpy(&build_status, status, 4, hipMemcpyDeviceToHost));
  if (build_status != MAP_OK || r.status != MAP_OK) {
    fprintf(stderr, "device status: build %d, detect %d\n", build_status, r.status);
    exit(2);
  }
  outcome o = {r.found, r.witness, r.iterations, -1, -1};
  if (r.found) {
    CHECK_MAP(map_lasso(n, row_ptr, col, r.witness, init, path, cap, d_lasso, ws, ws_bytes, NULL));
    map_lasso_result l;
    CHECK_HIP(hipMemcpy(&l, d_lasso, sizeof(l), hipMemcpyDeviceToHost));
    if (l.status != MAP_OK) {
      fprintf(stderr, "lasso status %d: %s\n", l.status, map_strerror(l.status));
      exit(2);
    }
    o.stem = l.stem_len;
    o.cycle = l.cycle_len;
  }
  hipFree(d_src); hipFree(d_dst); hipFree(d_acc); hipFree(row_ptr); hipFree(col); hipFree(status);
  hipFree(d_res); hipFree(d_lasso); hipFree(path); hipFree(ws);
  return o;
}

static int report(const char* name, outcome got, outcome want) {
  const int ok = memcmp(&got, &want, sizeof(got)) == 0;
  printf("%s: found %d witness %d K %d stem %d cycle %d %s\n", name, got.found, got.witness, got.iterations,
         got.stem, got.cycle, ok ? "ok" : "MISMATCH");
  return ok;
}

int main(void) {
  int ok = 1;
  {
    const int32_t src[] = {1, 2, 3, 3, 4}, dst[] = {2, 3, 1, 4, 5};
    const uint8_t acc[] = {0, 1, 0, 1, 1};
    const outcome want = {1, 2, 3, 1, 3};
    ok &= report("worked example", run(5, 5, src, dst, acc, 1), want);
  }
  {
    const int32_t n = 1000, ring = 600;
    int32_t* src = (int32_t*)malloc((size_t)n * 4);
    int32_t* dst = (int32_t*)malloc((size_t)n * 4);
    uint8_t* acc = (uint8_t*)calloc((size_t)n, 1);
    for (int32_t v = 1; v <= n; ++v) {
      src[v - 1] = v;
      dst[v - 1] = (v == ring || v == n) ? 1 : v + 1;  /* the ring closes at 600; the tail enters at 1 */
      acc[v - 1] = (v % 7 == 0);
    }
    const outcome want = {1, 595, 1, (n - (ring + 1)) + 1 + (595 - 1), ring};
    ok &= report("ring with tail", run(n, n, src, dst, acc, ring + 1), want);
    free(src); free(dst); free(acc);
  }
  return ok ? 0 : 1;
}

// Drives the C ABI's host-only calls (hss_plan_create / hss_plan_query /
// hss_plan_destroy, hss_default_opts, hss_last_error and the argument checks of
// hss_factor) on a structure read from a file, for a build with the host
// sanitizers. Prints, per box, "box <heap id> <height>" and the lines "I ...",
// "B ..." and "H ..." (interior dofs, boundary dofs, HSS tree as lo hi left right
// per node), then "R ..." (root dofs) and "ok".
//
// Input (little-endian int32): n_el q nnzb row_ptr[n_el+1] col_idx[nnzb]
// n_leaves leaf_node[n_leaves] leaf_ptr[n_leaves+1] leaf_elems[n_el] elem_xy[2 n_el]
// nheap heaps[nheap] leaf_size
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../include/hss.h"

static std::vector<int32_t> rd(FILE* f, size_t n) {
  std::vector<int32_t> v(n);
  if (n && std::fread(v.data(), 4, n, f) != n) {
    std::fprintf(stderr, "short input\n");
    std::exit(2);
  }
  return v;
}

static void put(const char* tag, const std::vector<int64_t>& v) {
  std::printf("%s", tag);
  for (int64_t x : v) std::printf(" %lld", (long long)x);
  std::printf("\n");
}

static std::vector<int64_t> query(hss_plan_t p, const char* key, int node) {
  int64_t len = 0;
  if (hss_plan_query(p, key, node, nullptr, 0, &len) != HSS_OK) {
    std::fprintf(stderr, "query %s %d: %s\n", key, node, hss_last_error());
    std::exit(3);
  }
  std::vector<int64_t> v((size_t)len);
  if (len && hss_plan_query(p, key, node, v.data(), len, &len) != HSS_OK) std::exit(3);
  return v;
}

int main(int argc, char** argv) {
  if (argc < 2) return 2;
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) return 2;
  auto hdr = rd(f, 3);
  const int n_el = hdr[0], q = hdr[1], nnzb = hdr[2];
  auto row_ptr = rd(f, (size_t)n_el + 1);
  auto col_idx = rd(f, (size_t)nnzb);
  const int n_leaves = rd(f, 1)[0];
  auto leaf_node = rd(f, (size_t)n_leaves);
  auto leaf_ptr = rd(f, (size_t)n_leaves + 1);
  auto leaf_elems = rd(f, (size_t)n_el);
  auto elem_xy = rd(f, 2 * (size_t)n_el);
  const int nheap = rd(f, 1)[0];
  auto heaps = rd(f, (size_t)nheap);
  const int leaf = rd(f, 1)[0];
  std::fclose(f);
  std::vector<double> vals((size_t)nnzb * q * q, 1.0);
  hss_block_op_t A{n_el, q, row_ptr.data(), col_idx.data(), vals.data(), HSS_R64, 0};
  hss_tree_t T{n_leaves, leaf_node.data(), leaf_ptr.data(), leaf_elems.data(), elem_xy.data()};
  hss_plan_t p = nullptr;
  if (hss_plan_create(&A, &T, leaf, &p) != HSS_OK) {
    std::fprintf(stderr, "plan: %s\n", hss_last_error());
    return 4;
  }
  for (int s : heaps) {
    std::printf("box %d %lld\n", s, (long long)query(p, "height", s)[0]);
    put("I", query(p, "idof", s));
    put("B", query(p, "bdof", s));
    put("H", query(p, "hss", s));
  }
  put("R", query(p, "root", 1));
  // error paths: unknown key and box, null arguments, a broken structure
  int64_t len = 0;
  if (hss_plan_query(p, "nope", heaps[0], nullptr, 0, &len) != HSS_EINVAL) return 5;
  if (hss_plan_query(p, "idof", 1 << 29, nullptr, 0, &len) != HSS_EINVAL) return 5;
  hss_plan_destroy(p);
  hss_plan_t p2 = nullptr;
  if (hss_plan_create(nullptr, &T, 0, &p2) == HSS_OK || p2) return 6;
  std::vector<int32_t> bad_ptr(row_ptr);
  bad_ptr[1] = bad_ptr[2] + 1;  // not monotone
  hss_block_op_t Ab = A;
  Ab.row_ptr = bad_ptr.data();
  if (hss_plan_create(&Ab, &T, 0, &p2) == HSS_OK || p2) return 6;
  if (hss_plan_create(&A, &T, -1, &p2) == HSS_OK || p2) return 6;
  // hss_factor's checks run before any device work; a NaN value is refused
  hss_opts_t o;
  hss_default_opts(&o);
  hss_handle_t h = nullptr;
  if (hss_factor(&A, &T, -1.0, &o, &h) != HSS_EINVAL || h) return 7;
  vals[0] = 0.0 / 0.0;
  if (hss_factor(&A, &T, 1e-4, &o, &h) != HSS_EINVAL || h) return 7;
  std::printf("ok\n");
  return 0;
}

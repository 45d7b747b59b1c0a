// Host-only driver of the analysis (analyze.cpp, graph_nd.cpp), for builds
// of those files under AddressSanitizer and UndefinedBehaviorSanitizer.  It
// is not part of libspaqr: the host sanitizer test compiles it with g++.
//
//   host_check <problems.bin> <out.bin>
//
// problems.bin (little-endian): int64 count, then per problem
//   int64 M, N, nnz; int32 grid[3], depth, skip, expect_error, in_union;
//   int64 row_ptr[M + 1]; int32 col_idx[nnz]; float64 vals[nnz]
// (a malformed problem may carry any row_ptr; nnz is the length of the
// arrays as stored).  Each problem is analysed on its own; the problems with
// in_union set are then joined into one block-diagonal plan.
//
// out.bin: per problem int32 status (0, or the error code thrown), then on
// success int32 column order [N] and int32 row owner [M] (finest-cluster
// index per row, the C-ABI's spaqr_get_ordering output); then the union's
// int32 status, int64 N, M and its column order and row owners.
// Exit status 0 when every problem did what expect_error says.
#include <cstdio>
#include <cstring>
#include <vector>

#include "spaqr_impl.h"

namespace {

template <typename T>
bool rd(std::FILE* f, T* p, size_t n) {
  return std::fread(p, sizeof(T), n, f) == n;
}

template <typename T>
void wr(std::FILE* f, const T* p, size_t n) {
  std::fwrite(p, sizeof(T), n, f);
}

void write_plan(std::FILE* o, const spaqr::Plan& P) {
  std::vector<int32_t> perm, owner((size_t)P.M);
  for (int c : P.finest)
    for (int j : P.clusters[c].cells) perm.push_back(j);
  for (int64_t r = 0; r < P.M; ++r) owner[r] = P.clusters[P.row_owner[r]].finest_index;
  wr(o, perm.data(), perm.size());
  wr(o, owner.data(), owner.size());
}

}  // namespace

int main(int argc, char** argv) {
  if (argc != 3) {
    std::fprintf(stderr, "usage: host_check <problems.bin> <out.bin>\n");
    return 2;
  }
  std::FILE* f = std::fopen(argv[1], "rb");
  std::FILE* o = std::fopen(argv[2], "wb");
  if (!f || !o) {
    std::fprintf(stderr, "cannot open the files\n");
    return 2;
  }
  int64_t count = 0;
  if (!rd(f, &count, 1) || count < 0) return 2;
  int bad = 0;
  std::vector<spaqr::Plan> parts;
  for (int64_t k = 0; k < count; ++k) {
    int64_t MNZ[3];
    int32_t hdr[7];
    if (!rd(f, MNZ, 3) || !rd(f, hdr, 7)) return 2;
    const int64_t M = MNZ[0], N = MNZ[1], nnz = MNZ[2];
    std::vector<int64_t> rp((size_t)std::max<int64_t>(M + 1, 0));
    std::vector<int32_t> ci((size_t)nnz);
    std::vector<double> va((size_t)nnz);
    if (!rd(f, rp.data(), rp.size()) || !rd(f, ci.data(), ci.size()) || !rd(f, va.data(), va.size())) return 2;
    spaqr_options opt{};
    for (int a = 0; a < 3; ++a) opt.grid[a] = hdr[a];
    opt.nd_depth = hdr[3];
    opt.sparsify_skip = hdr[4];
    opt.precision = SPAQR_FP64;
    const bool expect_error = hdr[5] != 0, in_union = hdr[6] != 0;
    spaqr::Plan P;
    int32_t status = 0;
    try {
      spaqr::analyze_plan(P, rp.data(), ci.data(), va.data(), M, N, opt);
    } catch (const spaqr::Error& e) {
      status = e.code;
    }
    wr(o, &status, 1);
    if (status == 0) write_plan(o, P);
    if ((status != 0) != expect_error) {
      std::fprintf(stderr, "problem %lld: status %d, expected %s\n", (long long)k, status,
                   expect_error ? "an error" : "success");
      ++bad;
    }
    if (status == 0 && in_union) parts.push_back(std::move(P));
  }
  spaqr::Plan U;
  int32_t status = 0;
  try {
    if (!parts.empty()) spaqr::union_plans(U, parts);
  } catch (const spaqr::Error& e) {
    status = e.code;
  }
  wr(o, &status, 1);
  const int64_t dims[2] = {U.N, U.M};
  wr(o, dims, 2);
  if (status == 0 && !parts.empty()) write_plan(o, U);
  std::fclose(f);
  std::fclose(o);
  return bad ? 1 : 0;
}

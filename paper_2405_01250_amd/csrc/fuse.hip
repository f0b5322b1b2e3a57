// fuse.hip -- DiaQ matrix product (Alg. 1) on the GPU: C = B * A.
//
// Alg. 1 pairs every diagonal a of one factor with every diagonal b of the
// other; the pair's element-wise product (the MultiplyDiagonals sub-kernel)
// lands on diagonal a + b.  Several pairs can land on the same diagonal, so
// their products are summed (the listing's plain assignment would keep only
// the last pair), and the sum runs in ascending a so the result does not
// depend on scheduling.  Each output element has one owning lane: no
// atomics on values, unlike the listing's parallel loop over diagonals.
//
// With C[i, i+c] = sum_{a+b=c} B[i, i+b] * A[i+b, i+c]: B's diagonal b is
// read at row i and A's diagonal a at row i + b.
#include <algorithm>
#include <map>

#include "internal.hpp"

namespace diaq {

namespace {

constexpr int kBlock = 256;

template <typename R>
struct Vec;
template <>
struct Vec<double> {
  using V = double2;
};
template <>
struct Vec<float> {
  using V = float2;
};

struct PairTerm {
  int64_t eb, vbb;  // B's diagonal index and value base (value at vbb + i)
  int64_t vba;      // A's value base (value at vba + m, m = i + eb)
};

struct OutDiag {
  int64_t c;      // output diagonal index
  int64_t start;  // packed start in the output buffer
  int32_t p0, np; // pair range
};

template <typename R>
__global__ __launch_bounds__(kBlock) void multiply_diagonals_kernel(
    int64_t N, const OutDiag* __restrict__ outs, const PairTerm* __restrict__ pairs,
    const typename Vec<R>::V* __restrict__ va, int conj_a, const typename Vec<R>::V* __restrict__ vb, int conj_b,
    double tol2, typename Vec<R>::V* __restrict__ out, int* __restrict__ flags) {
  using V = typename Vec<R>::V;
  const OutDiag od = outs[blockIdx.y];
  const int64_t len = N - (od.c < 0 ? -od.c : od.c);
  const int64_t t = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  bool nz = false;
  if (t < len) {
    const int64_t i = t + (od.c < 0 ? -od.c : 0);
    double ar = 0, ai = 0;
    for (int p = 0; p < od.np; p++) {
      const PairTerm pt = pairs[od.p0 + p];
      const int64_t m = i + pt.eb;
      if (m < 0 || m >= N) continue;  // B has no element in row i on diagonal b
      V b = vb[pt.vbb + i];
      V a = va[pt.vba + m];
      if (conj_b) b.y = -b.y;
      if (conj_a) a.y = -a.y;
      ar += double(b.x) * double(a.x) - double(b.y) * double(a.y);
      ai += double(b.x) * double(a.y) + double(b.y) * double(a.x);
    }
    const V cv = V{R(ar), R(ai)};
    out[od.start + t] = cv;
    // decided on the stored (possibly rounded-to-float) value
    const double sr = double(cv.x), si = double(cv.y);
    nz = (tol2 == 0.0) ? (sr != 0.0 || si != 0.0) : (sr * sr + si * si > tol2);
  }
  if (__any(nz) && (threadIdx.x & 63) == 0) atomicOr(&flags[blockIdx.y], 1);
}

// (applied diagonal index, value base) of stored diagonal kk under the
// operand's transpose flag: row i reads values[vb + i].
void applied(const diaq_dia* X, int kk, int64_t& e, int64_t& vbase) {
  const int64_t d = X->offsets[kk], st = X->starts[kk];
  if (X->transposed) {
    e = -d;
    vbase = st - (d > 0 ? d : 0);
  } else {
    e = d;
    vbase = st + (d < 0 ? d : 0);
  }
}

}  // namespace

diaq_status_t fuse_dia(diaq_ctx* ctx, const diaq_dia* A, const diaq_dia* B, double drop_tol, diaq_dia** out) {
  const int n = A->nqubits;
  const int64_t N = int64_t(1) << n;
  // group pairs by output index; within one output, ascending a
  std::map<int64_t, std::vector<PairTerm>> groups;
  std::vector<std::pair<int64_t, int>> aorder;
  for (int ka = 0; ka < A->ndiag; ka++) {
    int64_t ea, vba;
    applied(A, ka, ea, vba);
    aorder.push_back({ea, ka});
  }
  std::sort(aorder.begin(), aorder.end());
  for (auto& ao : aorder) {
    int64_t ea, vba;
    applied(A, ao.second, ea, vba);
    for (int kb = 0; kb < B->ndiag; kb++) {
      int64_t eb, vbb;
      applied(B, kb, eb, vbb);
      const int64_t c = ea + eb;
      if (c <= -N || c >= N) continue;
      // rows i of C's diagonal c with 0 <= i + eb < N
      const int64_t lo = std::max<int64_t>(c < 0 ? -c : 0, eb < 0 ? -eb : 0);
      const int64_t hi = std::min<int64_t>(c > 0 ? N - c : N, eb > 0 ? N - eb : N);
      if (lo >= hi) continue;
      groups[c].push_back(PairTerm{eb, vbb, vba});
    }
  }
  std::vector<OutDiag> outs;
  std::vector<PairTerm> pairs;
  std::vector<int64_t> coffs;
  int64_t total = 0;
  for (auto& g : groups) {
    OutDiag od;
    od.c = g.first;
    od.start = total;
    od.p0 = int32_t(pairs.size());
    od.np = int32_t(g.second.size());
    pairs.insert(pairs.end(), g.second.begin(), g.second.end());
    outs.push_back(od);
    coffs.push_back(g.first);
    total += N - (g.first < 0 ? -g.first : g.first);
  }
  if (outs.size() > 65535) return fail(DIAQ_ERR_UNSUPPORTED, "product has %zu diagonals", outs.size());
  const size_t eb = elem_bytes(A->dtype);
  // candidate result (kept as the output when no diagonal is dropped)
  diaq_dia* C = nullptr;
  DIAQ_TRY(new_dia(ctx, n, A->dtype, coffs, nullptr, false, &C));
  if (outs.empty()) {
    *out = C;
    return DIAQ_OK;
  }
  const size_t tbytes = outs.size() * sizeof(OutDiag) + pairs.size() * sizeof(PairTerm) + outs.size() * sizeof(int);
  diaq_status_t st = ensure(ctx, &ctx->aux, tbytes + 512);
  if (st != DIAQ_OK) {
    diaq_dia_free(C);
    return st;
  }
  char* base = static_cast<char*>(ctx->aux.ptr);
  OutDiag* douts = reinterpret_cast<OutDiag*>(base);
  PairTerm* dpairs = reinterpret_cast<PairTerm*>(base + ((outs.size() * sizeof(OutDiag) + 255) / 256) * 256);
  int* dflags = reinterpret_cast<int*>(reinterpret_cast<char*>(dpairs) +
                                       ((pairs.size() * sizeof(PairTerm) + 255) / 256) * 256);
  hipError_t he = hipMemcpyAsync(douts, outs.data(), outs.size() * sizeof(OutDiag), hipMemcpyHostToDevice, ctx->stream);
  if (he == hipSuccess)
    he = hipMemcpyAsync(dpairs, pairs.data(), pairs.size() * sizeof(PairTerm), hipMemcpyHostToDevice, ctx->stream);
  if (he == hipSuccess) he = hipMemsetAsync(dflags, 0, outs.size() * sizeof(int), ctx->stream);
  if (he != hipSuccess) {
    diaq_dia_free(C);
    return fail(DIAQ_ERR_DEVICE, "fuse table upload failed: %s", hipGetErrorString(he));
  }
  int64_t maxlen = 0;
  for (auto& od : outs) maxlen = std::max<int64_t>(maxlen, N - (od.c < 0 ? -od.c : od.c));
  dim3 grid(unsigned((maxlen + kBlock - 1) / kBlock), unsigned(outs.size()));
  const double tol2 = drop_tol * drop_tol;
  if (A->dtype == DIAQ_C128)
    hipLaunchKernelGGL(multiply_diagonals_kernel<double>, grid, dim3(kBlock), 0, ctx->stream, N, douts, dpairs,
                       static_cast<const double2*>(A->values), A->conjugated ? 1 : 0,
                       static_cast<const double2*>(B->values), B->conjugated ? 1 : 0, tol2,
                       static_cast<double2*>(C->values), dflags);
  else
    hipLaunchKernelGGL(multiply_diagonals_kernel<float>, grid, dim3(kBlock), 0, ctx->stream, N, douts, dpairs,
                       static_cast<const float2*>(A->values), A->conjugated ? 1 : 0,
                       static_cast<const float2*>(B->values), B->conjugated ? 1 : 0, tol2,
                       static_cast<float2*>(C->values), dflags);
  he = hipGetLastError();
  std::vector<int> flags(outs.size(), 0);
  if (he == hipSuccess) he = hipMemcpyAsync(flags.data(), dflags, flags.size() * sizeof(int), hipMemcpyDeviceToHost, ctx->stream);
  if (he == hipSuccess) he = hipStreamSynchronize(ctx->stream);
  if (he != hipSuccess) {
    diaq_dia_free(C);
    return fail(DIAQ_ERR_DEVICE, "fuse kernel failed: %s", hipGetErrorString(he));
  }
  std::vector<int64_t> kept;
  std::vector<size_t> kept_idx;
  for (size_t q = 0; q < outs.size(); q++)
    if (flags[q]) {
      kept.push_back(outs[q].c);
      kept_idx.push_back(q);
    }
  if (kept.size() == outs.size()) {
    C->qubit_mask = A->qubit_mask | B->qubit_mask;
    *out = C;
    return DIAQ_OK;
  }
  diaq_dia* D = nullptr;
  st = new_dia(ctx, n, A->dtype, kept, nullptr, false, &D);
  if (st != DIAQ_OK) {
    diaq_dia_free(C);
    return st;
  }
  for (size_t q = 0; q < kept.size(); q++) {
    const OutDiag& od = outs[kept_idx[q]];
    const int64_t len = N - (od.c < 0 ? -od.c : od.c);
    he = hipMemcpyAsync(static_cast<char*>(D->values) + size_t(D->starts[q]) * eb,
                        static_cast<const char*>(C->values) + size_t(od.start) * eb, size_t(len) * eb,
                        hipMemcpyDeviceToDevice, ctx->stream);
    if (he != hipSuccess) break;
  }
  if (he == hipSuccess) he = hipStreamSynchronize(ctx->stream);
  diaq_dia_free(C);
  if (he != hipSuccess) {
    diaq_dia_free(D);
    return fail(DIAQ_ERR_DEVICE, "fuse compaction failed: %s", hipGetErrorString(he));
  }
  D->qubit_mask = A->qubit_mask | B->qubit_mask;
  *out = D;
  return DIAQ_OK;
}

}  // namespace diaq

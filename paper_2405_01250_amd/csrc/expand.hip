// expand.hip -- writes the DiaQ diagonals of an expanded gate (the time-step
// unitary I_above (x) Gate (x) I_below of Sec. II-C) and of Pauli sums.
//
// Expansion is a pure write stream (Sec. VI notes the Kronecker step needs
// almost no arithmetic): element t of diagonal d is A[i, i + d] with
// i = t + max(0, -d).  One workgroup row covers one diagonal; each lane
// writes 16-byte (c128) elements, consecutive lanes consecutive elements.
#include "internal.hpp"

namespace diaq {

namespace {

constexpr int kBlock = 256;
// Pauli-sum diagonals: one element per lane (several elements per lane a
// block apart measured slower for this write stream).
constexpr int kPerThread = 1;

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

struct ExpandArgs {
  int64_t N;
  int32_t nd;
  int32_t k;
  int32_t targets[3];
  int32_t pad;
  uint64_t tmask;
  uint64_t cmask;
  int64_t off[kMaxArgDiags];
  int64_t start[kMaxArgDiags];
  double m[8][8][2];
  const char* tabs;  // diagonal gates applied after the core (factor tables)
  int32_t nt;
  int32_t pad2;
};

template <bool NT, typename V>
__device__ __forceinline__ void put(V* p, const V& v) {
  if constexpr (NT) {
    using N2 = typename HIP_vector_base<decltype(V{}.x), 2>::Native_vec_;
    N2 t = {v.x, v.y};
    __builtin_nontemporal_store(t, reinterpret_cast<N2*>(p));
  } else {
    *p = v;
  }
}

// Element t of diagonal d (row i = t + max(0, -d), column j = i + d) of the
// expanded gate, times the folded diagonal factors of row i.
__device__ __forceinline__ void expanded_element(const ExpandArgs& a, const double (*sm)[2], int dim, int64_t d,
                                                 int64_t row0, int64_t t, double& vr, double& vi) {
  const uint64_t i = uint64_t(t + row0);
  const uint64_t j = uint64_t(int64_t(i) + d);
  vr = 0;
  vi = 0;
  if (((i ^ j) & ~a.tmask) == 0) {
    if ((i & a.cmask) != a.cmask) {
      vr = (i == j) ? 1.0 : 0.0;
    } else {
      int r = 0, c = 0;
      for (int b = 0; b < a.k; b++) {
        r |= int((i >> a.targets[b]) & 1) << b;
        c |= int((j >> a.targets[b]) & 1) << b;
      }
      vr = sm[r * dim + c][0];
      vi = sm[r * dim + c][1];
    }
  }
  // folded diagonal gates D after the core: (D A)[i, j] = D(i) A[i, j]
  if (a.nt) apply_tables(a.tabs, a.nt, i, vr, vi);
}

// One lane per element for complex128 (16-byte stores); two consecutive
// elements per lane for complex64, stored as one 16-byte write when the pair
// is 16-byte aligned.
template <typename R, bool NT>
__global__ __launch_bounds__(kBlock) void expand_kernel(ExpandArgs a, typename Vec<R>::V* __restrict__ out) {
  using V = typename Vec<R>::V;
  constexpr int EPL = sizeof(R) == 4 ? 2 : 1;
  __shared__ double sm[64][2];
  const int dim = 1 << a.k;
  for (int t = threadIdx.x; t < dim * dim; t += kBlock) {
    sm[t][0] = a.m[t / dim][t % dim][0];
    sm[t][1] = a.m[t / dim][t % dim][1];
  }
  __syncthreads();
  const int kd = blockIdx.y;
  const int64_t d = a.off[kd];
  const int64_t len = a.N - (d < 0 ? -d : d);
  const int64_t row0 = d < 0 ? -d : 0;
  V* dst = out + a.start[kd];
  const int64_t t0 = (int64_t(blockIdx.x) * kBlock + threadIdx.x) * EPL;
  if (t0 >= len) return;
  double vr[EPL], vi[EPL];
#pragma unroll
  for (int e = 0; e < EPL; e++)
    if (t0 + e < len) expanded_element(a, sm, dim, d, row0, t0 + e, vr[e], vi[e]);
  if constexpr (EPL == 2) {
    if (t0 + 1 < len && ((a.start[kd] + t0) & 1) == 0) {
      const float4 w{float(vr[0]), float(vi[0]), float(vr[1]), float(vi[1])};
      *reinterpret_cast<float4*>(dst + t0) = w;
      return;
    }
  }
#pragma unroll
  for (int e = 0; e < EPL; e++)
    if (t0 + e < len) put<NT>(dst + t0 + e, V{R(vr[e]), R(vi[e])});
}

// Pauli-sum diagonals: element (i, j) = sum over terms with x == i ^ j of
// coef * i^{|x & z|} * (-1)^{|j & z|}.
struct PauliTerm {
  uint64_t x, z;
  double coef;
};

template <typename R>
__global__ __launch_bounds__(kBlock) void pauli_kernel(int64_t N, const int64_t* __restrict__ offs,
                                                       const int64_t* __restrict__ starts,
                                                       const PauliTerm* __restrict__ terms, int nterms,
                                                       typename Vec<R>::V* __restrict__ out) {
  using V = typename Vec<R>::V;
  const int kd = blockIdx.y;
  const int64_t d = offs[kd];
  const int64_t len = N - (d < 0 ? -d : d);
  const int64_t row0 = d < 0 ? -d : 0;
  V* dst = out + starts[kd];
  const int64_t t0 = int64_t(blockIdx.x) * (kBlock * kPerThread) + threadIdx.x;
#pragma unroll
  for (int e = 0; e < kPerThread; e++) {
    const int64_t t = t0 + e * kBlock;
    if (t >= len) break;
    const uint64_t i = uint64_t(t + row0);
    const uint64_t j = uint64_t(int64_t(i) + d);
    const uint64_t flip = i ^ j;
    double vr = 0, vi = 0;
    for (int q = 0; q < nterms; q++) {
      const PauliTerm tm = terms[q];
      if (tm.x != flip) continue;
      const int ny = __popcll(tm.x & tm.z) & 3;
      const double sg = (__popcll(j & tm.z) & 1) ? -1.0 : 1.0;
      // i^ny: 1, i, -1, -i
      const double pr = (ny == 0) ? 1.0 : (ny == 2) ? -1.0 : 0.0;
      const double pi = (ny == 1) ? 1.0 : (ny == 3) ? -1.0 : 0.0;
      vr += tm.coef * sg * pr;
      vi += tm.coef * sg * pi;
    }
    dst[t] = V{R(vr), R(vi)};
  }
}

}  // namespace

diaq_status_t launch_expand(diaq_ctx* ctx, const LocalGate& lg, int n, diaq_dtype_t dt,
                            const std::vector<int64_t>& offs, const std::vector<int64_t>& starts, void* values,
                            const void* tabs, int ntabs) {
  if (offs.size() > size_t(kMaxArgDiags))
    return fail(DIAQ_ERR_INVALID_ARGUMENT, "gate occupies %zu diagonals (> %d)", offs.size(), kMaxArgDiags);
  if (offs.empty()) return DIAQ_OK;
  ExpandArgs a;
  std::memset(&a, 0, sizeof(a));
  a.N = int64_t(1) << n;
  a.nd = int32_t(offs.size());
  a.k = lg.k;
  for (int j = 0; j < lg.k; j++) a.targets[j] = lg.targets[j];
  a.tmask = lg.tmask;
  a.cmask = lg.cmask;
  a.tabs = static_cast<const char*>(tabs);
  a.nt = tabs ? ntabs : 0;
  int64_t maxlen = 0;
  for (size_t q = 0; q < offs.size(); q++) {
    a.off[q] = offs[q];
    a.start[q] = starts[q];
    maxlen = std::max<int64_t>(maxlen, a.N - (offs[q] < 0 ? -offs[q] : offs[q]));
  }
  std::memcpy(a.m, lg.m, sizeof(a.m));
  const int64_t per_block = int64_t(kBlock) * (dt == DIAQ_C64 ? 2 : 1);
  const int64_t gx = (maxlen + per_block - 1) / per_block;
  dim3 grid(unsigned(gx), unsigned(offs.size()));
  // default: non-temporal stores for complex64 (measured 6.1 -> 6.5 TB/s at
  // n = 28), plain ones for complex128 (6.83 against 6.76 TB/s)
  const int32_t knob = ctx->tuning.expand_nontemporal;
  const bool nt = knob > 0 || (knob == 0 && dt == DIAQ_C64);
  if (dt == DIAQ_C128) {
    if (nt)
      hipLaunchKernelGGL((expand_kernel<double, true>), grid, dim3(kBlock), 0, ctx->stream, a,
                         static_cast<double2*>(values));
    else
      hipLaunchKernelGGL((expand_kernel<double, false>), grid, dim3(kBlock), 0, ctx->stream, a,
                         static_cast<double2*>(values));
  } else {
    if (nt)
      hipLaunchKernelGGL((expand_kernel<float, true>), grid, dim3(kBlock), 0, ctx->stream, a,
                         static_cast<float2*>(values));
    else
      hipLaunchKernelGGL((expand_kernel<float, false>), grid, dim3(kBlock), 0, ctx->stream, a,
                         static_cast<float2*>(values));
  }
  DIAQ_HIP(hipGetLastError());
  return DIAQ_OK;
}

diaq_status_t launch_pauli_dia(diaq_ctx* ctx, int n, diaq_dtype_t dt, const std::vector<int64_t>& offs,
                               const std::vector<int64_t>& starts, const uint64_t* xm, const uint64_t* zm,
                               const double* coef, int nterms, void* values) {
  if (offs.empty()) return DIAQ_OK;
  const int64_t N = int64_t(1) << n;
  std::vector<PauliTerm> terms(nterms);
  for (int q = 0; q < nterms; q++) terms[q] = PauliTerm{xm[q], zm[q], coef[q]};
  const size_t tb = offs.size() * sizeof(int64_t) * 2 + sizeof(int64_t) + terms.size() * sizeof(PauliTerm);
  DIAQ_TRY(ensure(ctx, &ctx->aux, tb + 256));
  char* base = static_cast<char*>(ctx->aux.ptr);
  int64_t* doffs = reinterpret_cast<int64_t*>(base);
  int64_t* dstarts = doffs + offs.size();
  PauliTerm* dterms = reinterpret_cast<PauliTerm*>(dstarts + offs.size() + 1);
  DIAQ_HIP(hipMemcpyAsync(doffs, offs.data(), offs.size() * sizeof(int64_t), hipMemcpyHostToDevice, ctx->stream));
  DIAQ_HIP(hipMemcpyAsync(dstarts, starts.data(), starts.size() * sizeof(int64_t), hipMemcpyHostToDevice,
                          ctx->stream));
  if (nterms)
    DIAQ_HIP(hipMemcpyAsync(dterms, terms.data(), terms.size() * sizeof(PauliTerm), hipMemcpyHostToDevice,
                            ctx->stream));
  int64_t maxlen = 0;
  for (int64_t d : offs) maxlen = std::max<int64_t>(maxlen, N - (d < 0 ? -d : d));
  const int64_t gx = (maxlen + kBlock * kPerThread - 1) / (kBlock * kPerThread);
  if (offs.size() > 65535) return fail(DIAQ_ERR_UNSUPPORTED, "Pauli sum with %zu diagonals", offs.size());
  dim3 grid(unsigned(gx), unsigned(offs.size()));
  if (dt == DIAQ_C128)
    hipLaunchKernelGGL(pauli_kernel<double>, grid, dim3(kBlock), 0, ctx->stream, N, doffs, dstarts, dterms, nterms,
                       static_cast<double2*>(values));
  else
    hipLaunchKernelGGL(pauli_kernel<float>, grid, dim3(kBlock), 0, ctx->stream, N, doffs, dstarts, dterms, nterms,
                       static_cast<float2*>(values));
  DIAQ_HIP(hipGetLastError());
  // the host vectors die on return: wait for the copies to finish reading them
  DIAQ_HIP(hipStreamSynchronize(ctx->stream));
  return DIAQ_OK;
}

}  // namespace diaq

// chain.hip -- matrix-level simulation on DiaQ matrices: unitary simulation
// (the product of all time-step unitaries of a circuit, Sec. II-A, with the
// per-step diagonal count and sparsity the paper tracks in Sec. III-A) and
// density-matrix evolution rho <- G rho G^dagger (Sec. II-A), both built
// from the Alg. 1 product (fuse_dia) and the free transpose of Sec. IV.
//
// Also: the number of stored non-zeros of a DiaQ matrix, and Tr(A B)
// (expectation values Tr(H rho) and the purity Tr(rho^2)).
#include <algorithm>
#include <new>

#include "internal.hpp"

namespace diaq {

namespace {

constexpr int kBlock = 256;
constexpr int kTraceBlocks = 1024;

template <typename R>
__global__ __launch_bounds__(kBlock) void nnz_kernel(const typename Cx<R>::V* __restrict__ v, int64_t count,
                                                     double tol2, unsigned long long* __restrict__ total) {
  unsigned long long c = 0;
  const int64_t stride = int64_t(gridDim.x) * kBlock;
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < count; i += stride) {
    const double re = double(v[i].x), im = double(v[i].y);
    c += (tol2 == 0.0) ? (re != 0.0 || im != 0.0) : (re * re + im * im > tol2);
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off, 64);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(total, c);
}

template <typename R>
__global__ __launch_bounds__(kBlock) void fill_one_kernel(typename Cx<R>::V* __restrict__ v, int64_t count) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i < count) v[i] = typename Cx<R>::V{R(1), R(0)};
}

// One term of Tr(A B): A's applied diagonal d against B's applied diagonal
// -d.  Row i of the term reads A[i, i+d] at va + i and B[i+d, i] at
// vb + i (bases already shifted); rows run over [lo, lo + len).
struct TraceTerm {
  int64_t va, vb, lo, len, prefix;  // prefix: first flattened index
  int32_t conj_a, conj_b;
};

template <typename R>
__global__ __launch_bounds__(kBlock) void trace_product_kernel(const TraceTerm* __restrict__ terms, int nterms,
                                                               int64_t total, const typename Cx<R>::V* __restrict__ a,
                                                               const typename Cx<R>::V* __restrict__ b,
                                                               double2* __restrict__ partial) {
  double re = 0, im = 0;
  const int64_t stride = int64_t(gridDim.x) * kBlock;
  for (int64_t f = int64_t(blockIdx.x) * kBlock + threadIdx.x; f < total; f += stride) {
    int lo = 0, hi = nterms - 1;  // last term with prefix <= f
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (terms[mid].prefix <= f) lo = mid;
      else hi = mid - 1;
    }
    const TraceTerm t = terms[lo];
    const int64_t i = t.lo + (f - t.prefix);
    const double ar = double(a[t.va + i].x), ai = t.conj_a ? -double(a[t.va + i].y) : double(a[t.va + i].y);
    const double br = double(b[t.vb + i].x), bi = t.conj_b ? -double(b[t.vb + i].y) : double(b[t.vb + i].y);
    re += ar * br - ai * bi;
    im += ar * bi + ai * br;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    re += __shfl_xor(re, off, 64);
    im += __shfl_xor(im, off, 64);
  }
  __shared__ double2 ws[kBlock / 64];
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = double2{re, im};
  __syncthreads();
  if (threadIdx.x == 0) {
    double2 s = ws[0];
    for (int w = 1; w < kBlock / 64; w++) {
      s.x += ws[w].x;
      s.y += ws[w].y;
    }
    partial[blockIdx.x] = s;
  }
}

// Applied diagonal index of stored diagonal k (the transpose flag negates
// it) and the value base such that row i of the applied matrix reads
// values[base + i].
void applied_diag(const diaq_dia* X, int k, int64_t& e, int64_t& base) {
  const int64_t d = X->offsets[k], st = X->starts[k];
  if (X->transposed) {
    e = -d;
    base = st - (d > 0 ? d : 0);
  } else {
    e = d;
    base = st + (d < 0 ? d : 0);
  }
}

int64_t stored_count(const diaq_dia* A) { return A->starts.empty() ? 0 : A->starts.back(); }

diaq_status_t count_nnz(diaq_ctx* ctx, const diaq_dia* A, double tol, int64_t* nnz) {
  const int64_t E = stored_count(A);
  DIAQ_TRY(ensure(ctx, &ctx->aux, 256));
  unsigned long long* dcount = static_cast<unsigned long long*>(ctx->aux.ptr);
  DIAQ_HIP(hipMemsetAsync(dcount, 0, sizeof(unsigned long long), ctx->stream));
  if (E > 0) {
    const int64_t want = (E + kBlock - 1) / kBlock;
    const unsigned blocks = unsigned(std::min<int64_t>(want, int64_t(ctx->num_cus) * 16));
    const double tol2 = tol * tol;
    if (A->dtype == DIAQ_C128)
      hipLaunchKernelGGL(nnz_kernel<double>, dim3(blocks), dim3(kBlock), 0, ctx->stream,
                         static_cast<const double2*>(A->values), E, tol2, dcount);
    else
      hipLaunchKernelGGL(nnz_kernel<float>, dim3(blocks), dim3(kBlock), 0, ctx->stream,
                         static_cast<const float2*>(A->values), E, tol2, dcount);
    DIAQ_HIP(hipGetLastError());
  }
  DIAQ_TRY(ensure_pinned(ctx, sizeof(double)));
  DIAQ_HIP(hipMemcpyAsync(ctx->pinned, dcount, sizeof(unsigned long long), hipMemcpyDeviceToHost, ctx->stream));
  DIAQ_HIP(hipStreamSynchronize(ctx->stream));
  unsigned long long c;
  std::memcpy(&c, ctx->pinned, sizeof(c));
  *nnz = int64_t(c);
  return DIAQ_OK;
}

diaq_status_t record_step(diaq_ctx* ctx, const diaq_dia* U, double tol, diaq_chain_step_t* step) {
  if (!step) return DIAQ_OK;
  step->ndiag = U->ndiag;
  step->reserved = 0;
  step->nvalues = stored_count(U);
  return count_nnz(ctx, U, tol, &step->nnz);
}

diaq_status_t identity(diaq_ctx* ctx, int n, diaq_dtype_t dt, diaq_dia** out) {
  diaq_dia* I = nullptr;
  DIAQ_TRY(new_dia(ctx, n, dt, std::vector<int64_t>{0}, nullptr, false, &I));
  const int64_t N = int64_t(1) << n;
  const unsigned blocks = unsigned((N + kBlock - 1) / kBlock);
  if (dt == DIAQ_C128)
    hipLaunchKernelGGL(fill_one_kernel<double>, dim3(blocks), dim3(kBlock), 0, ctx->stream,
                       static_cast<double2*>(I->values), N);
  else
    hipLaunchKernelGGL(fill_one_kernel<float>, dim3(blocks), dim3(kBlock), 0, ctx->stream,
                       static_cast<float2*>(I->values), N);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    diaq_dia_free(I);
    return fail(DIAQ_ERR_DEVICE, "identity fill failed: %s", hipGetErrorString(e));
  }
  I->qubit_mask = 0;
  *out = I;
  return DIAQ_OK;
}

// A copy that owns its values, with the transpose / conjugate flags of X
// folded in by a product with the identity (first = X, second = I).
diaq_status_t owned_copy(diaq_ctx* ctx, const diaq_dia* X, diaq_dia** out) {
  diaq_dia* I = nullptr;
  DIAQ_TRY(identity(ctx, X->nqubits, X->dtype, &I));
  const diaq_status_t st = fuse_dia(ctx, X, I, 0.0, out);
  diaq_dia_free(I);
  return st;
}

diaq_status_t expand_gate(diaq_ctx* ctx, const diaq_gate_t* g, int n, diaq_dtype_t dt, diaq_dia** out) {
  LocalGate lg;
  DIAQ_TRY(local_gate(g, n, &lg));
  diaq_dia* G = nullptr;
  DIAQ_TRY(new_dia(ctx, n, dt, gate_offsets(lg), nullptr, false, &G));
  G->qubit_mask = lg.tmask;
  const diaq_status_t st = launch_expand(ctx, lg, n, dt, G->offsets, G->starts, G->values);
  if (st != DIAQ_OK) {
    diaq_dia_free(G);
    return st;
  }
  *out = G;
  return DIAQ_OK;
}

// Replace *cur by next (freeing the old one).
void advance(diaq_dia** cur, diaq_dia* next) {
  diaq_dia_free(*cur);
  *cur = next;
}

diaq_status_t check_gates(const diaq_gate_t* gates, int64_t ngates, int n) {
  if (ngates < 0 || (ngates > 0 && !gates)) return fail(DIAQ_ERR_INVALID_ARGUMENT, "bad gate list");
  for (int64_t t = 0; t < ngates; t++) {
    LocalGate lg;
    const diaq_status_t st = local_gate(&gates[t], n, &lg);
    if (st != DIAQ_OK) return st;
  }
  return DIAQ_OK;
}

}  // namespace

}  // namespace diaq

using namespace diaq;

extern "C" {

diaq_status_t diaq_dia_nnz(diaq_ctx_t ctx, diaq_dia_t A, double tol, int64_t* nnz) {
  try {
    if (!ctx || !A || !nnz) return fail(DIAQ_ERR_INVALID_ARGUMENT, "NULL argument");
    if (!(tol >= 0)) return fail(DIAQ_ERR_INVALID_ARGUMENT, "tol must be >= 0");
    return count_nnz(ctx, A, tol, nnz);
  } catch (const std::bad_alloc&) {
    return fail(DIAQ_ERR_OUT_OF_MEMORY, "host allocation failed");
  }
}

diaq_status_t diaq_trace_product(diaq_ctx_t ctx, diaq_dia_t A, diaq_dia_t B, double* out) {
  try {
    if (!ctx || !A || !B || !out) return fail(DIAQ_ERR_INVALID_ARGUMENT, "NULL argument");
    if (A->nqubits != B->nqubits || A->dtype != B->dtype)
      return fail(DIAQ_ERR_NOT_MULTIPLYABLE, "not multiplyable: 2^%d vs 2^%d", A->nqubits, B->nqubits);
    const int64_t N = int64_t(1) << A->nqubits;
    // B's applied diagonals by index
    std::vector<std::pair<int64_t, int64_t>> bd(B->ndiag);
    for (int k = 0; k < B->ndiag; k++) applied_diag(B, k, bd[k].first, bd[k].second);
    std::sort(bd.begin(), bd.end());
    std::vector<std::pair<int64_t, int>> ad(A->ndiag);
    for (int k = 0; k < A->ndiag; k++) {
      int64_t e, base;
      applied_diag(A, k, e, base);
      ad[k] = {e, k};
    }
    std::sort(ad.begin(), ad.end());
    std::vector<TraceTerm> terms;
    int64_t total = 0;
    for (auto& p : ad) {
      int64_t d, va;
      applied_diag(A, p.second, d, va);
      auto it = std::lower_bound(bd.begin(), bd.end(), std::make_pair(-d, INT64_MIN));
      if (it == bd.end() || it->first != -d) continue;
      // rows i with A[i, i+d] and B[i+d, i] both inside the matrix
      const int64_t lo = d < 0 ? -d : 0, hi = d > 0 ? N - d : N;
      if (lo >= hi) continue;
      TraceTerm t;
      t.va = va;
      t.vb = it->second + d;  // B's row i + d
      t.lo = lo;
      t.len = hi - lo;
      t.prefix = total;
      t.conj_a = A->conjugated ? 1 : 0;
      t.conj_b = B->conjugated ? 1 : 0;
      terms.push_back(t);
      total += t.len;
    }
    if (terms.empty()) {
      out[0] = out[1] = 0.0;
      return DIAQ_OK;
    }
    const size_t tbytes = ((terms.size() * sizeof(TraceTerm) + 255) / 256) * 256;
    DIAQ_TRY(ensure(ctx, &ctx->aux, tbytes + 2 * sizeof(double) + 256));
    DIAQ_TRY(ensure(ctx, &ctx->red, kTraceBlocks * sizeof(double2)));
    TraceTerm* dterms = static_cast<TraceTerm*>(ctx->aux.ptr);
    double* dres = reinterpret_cast<double*>(static_cast<char*>(ctx->aux.ptr) + tbytes);
    double2* partial = static_cast<double2*>(ctx->red.ptr);
    DIAQ_HIP(hipMemcpyAsync(dterms, terms.data(), terms.size() * sizeof(TraceTerm), hipMemcpyHostToDevice,
                            ctx->stream));
    if (A->dtype == DIAQ_C128)
      hipLaunchKernelGGL(trace_product_kernel<double>, dim3(kTraceBlocks), dim3(kBlock), 0, ctx->stream, dterms,
                         int(terms.size()), total, static_cast<const double2*>(A->values),
                         static_cast<const double2*>(B->values), partial);
    else
      hipLaunchKernelGGL(trace_product_kernel<float>, dim3(kTraceBlocks), dim3(kBlock), 0, ctx->stream, dterms,
                         int(terms.size()), total, static_cast<const float2*>(A->values),
                         static_cast<const float2*>(B->values), partial);
    DIAQ_HIP(hipGetLastError());
    DIAQ_TRY(launch_final_reduce(ctx->stream, partial, kTraceBlocks, dres));
    DIAQ_TRY(ensure_pinned(ctx, 2 * sizeof(double)));
    DIAQ_HIP(hipMemcpyAsync(ctx->pinned, dres, 2 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    DIAQ_HIP(hipStreamSynchronize(ctx->stream));
    out[0] = ctx->pinned[0];
    out[1] = ctx->pinned[1];
    return DIAQ_OK;
  } catch (const std::bad_alloc&) {
    return fail(DIAQ_ERR_OUT_OF_MEMORY, "host allocation failed");
  }
}

diaq_status_t diaq_unitary(diaq_ctx_t ctx, const diaq_gate_t* gates, int64_t ngates, int32_t nqubits,
                           diaq_dtype_t dtype, diaq_dia_t start, double drop_tol, diaq_chain_step_t* steps,
                           diaq_dia_t* out) {
  try {
    if (!ctx || !out) return fail(DIAQ_ERR_INVALID_ARGUMENT, "ctx/out is NULL");
    if (dtype != DIAQ_C64 && dtype != DIAQ_C128) return fail(DIAQ_ERR_INVALID_ARGUMENT, "bad dtype");
    if (nqubits < 1 || nqubits > 15)
      return fail(DIAQ_ERR_UNSUPPORTED, "unitary simulation holds 2^n x 2^n matrices; n = %d outside [1, 15]",
                  nqubits);
    if (!(drop_tol >= 0)) return fail(DIAQ_ERR_INVALID_ARGUMENT, "drop_tol must be >= 0");
    if (start && (start->nqubits != nqubits || start->dtype != dtype))
      return fail(DIAQ_ERR_NOT_MULTIPLYABLE, "start matrix does not match n / dtype");
    DIAQ_TRY(check_gates(gates, ngates, nqubits));
    diaq_dia* U = nullptr;
    DIAQ_TRY(start ? owned_copy(ctx, start, &U) : identity(ctx, nqubits, dtype, &U));
    for (int64_t t = 0; t < ngates; t++) {
      diaq_dia* G = nullptr;
      diaq_status_t st = expand_gate(ctx, &gates[t], nqubits, dtype, &G);
      diaq_dia* next = nullptr;
      if (st == DIAQ_OK) st = fuse_dia(ctx, U, G, drop_tol, &next);  // G * U
      diaq_dia_free(G);
      if (st == DIAQ_OK) {
        advance(&U, next);
        st = record_step(ctx, U, drop_tol, steps ? &steps[t] : nullptr);
      }
      if (st != DIAQ_OK) {
        diaq_dia_free(U);
        return st;
      }
    }
    *out = U;
    return DIAQ_OK;
  } catch (const std::bad_alloc&) {
    return fail(DIAQ_ERR_OUT_OF_MEMORY, "host allocation failed");
  }
}

diaq_status_t diaq_density_evolve(diaq_ctx_t ctx, const diaq_gate_t* gates, int64_t ngates, diaq_dia_t rho,
                                  double drop_tol, diaq_chain_step_t* steps, diaq_dia_t* out) {
  try {
    if (!ctx || !rho || !out) return fail(DIAQ_ERR_INVALID_ARGUMENT, "NULL argument");
    const int n = rho->nqubits;
    if (n > 15) return fail(DIAQ_ERR_UNSUPPORTED, "density matrices are 2^n x 2^n; n = %d above 15", n);
    if (!(drop_tol >= 0)) return fail(DIAQ_ERR_INVALID_ARGUMENT, "drop_tol must be >= 0");
    DIAQ_TRY(check_gates(gates, ngates, n));
    diaq_dia* R = nullptr;
    DIAQ_TRY(owned_copy(ctx, rho, &R));
    for (int64_t t = 0; t < ngates; t++) {
      diaq_dia* G = nullptr;
      diaq_status_t st = expand_gate(ctx, &gates[t], n, rho->dtype, &G);
      diaq_dia* left = nullptr;
      if (st == DIAQ_OK) st = fuse_dia(ctx, R, G, drop_tol, &left);  // G * rho
      if (st == DIAQ_OK) {
        // G^dagger: the transpose is a relabelling of G's diagonals and
        // the conjugation a flag on its values (Sec. IV)
        diaq_dia Gd = *G;
        Gd.owns_values = false;
        Gd.dmeta = nullptr;
        Gd.transposed = !G->transposed;
        Gd.conjugated = !G->conjugated;
        diaq_dia* next = nullptr;
        st = fuse_dia(ctx, &Gd, left, drop_tol, &next);  // (G rho) * G^dagger
        diaq_dia_free(left);
        if (st == DIAQ_OK) advance(&R, next);
      }
      diaq_dia_free(G);
      if (st == DIAQ_OK) st = record_step(ctx, R, drop_tol, steps ? &steps[t] : nullptr);
      if (st != DIAQ_OK) {
        diaq_dia_free(R);
        return st;
      }
    }
    *out = R;
    return DIAQ_OK;
  } catch (const std::bad_alloc&) {
    return fail(DIAQ_ERR_OUT_OF_MEMORY, "host allocation failed");
  }
}

}  // extern "C"

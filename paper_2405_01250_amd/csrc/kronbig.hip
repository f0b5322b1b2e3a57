// kronbig.hip -- Alg. 3 with fused groups of up to five qubits.
//
// On the in-place (Alg. 3) path an operation costs one read and one write of
// the state whatever its matrix, so fusing more gates into fewer operations
// is pure gain as long as the arithmetic stays under the memory time.  The
// planner here groups gates the same way as the three-qubit planner (a gate
// joins the latest operation that shares a qubit, which it may move past
// because it commutes with everything after it) but lets a group span up to
// five qubits, multiplying the gates' embedded matrices into one dense
// 2^k x 2^k matrix (controls are qubits of the group).  Diagonal gates that
// do not fit stay row factors of an operation.  A lane owns one coset of the
// group (Alg. 3's cosets), keeps its 2^k amplitudes in registers, reads the
// matrix from LDS and writes each output row as soon as it is formed.
#include <complex>

#include "internal.hpp"

namespace diaq {

namespace {

using Cd = std::complex<double>;
constexpr int kBigBlock = 256;
constexpr int kBigMaxFactors = 64;

// Matrix of gate lg on the group qubits S (bit j of a local index is S[j]):
// P_ctrl (x) M + (1 - P_ctrl) (x) 1, identity on the group's other qubits.
std::vector<Cd> embed_gate(const LocalGate& lg, const int* S, int k) {
  const int D = 1 << k;
  auto pos = [&](int q) {
    for (int j = 0; j < k; j++)
      if (S[j] == q) return j;
    return -1;
  };
  int tpos[3], cpos[3];
  uint32_t tm = 0;
  for (int j = 0; j < lg.k; j++) {
    tpos[j] = pos(lg.targets[j]);
    tm |= 1u << tpos[j];
  }
  for (int j = 0; j < lg.nc; j++) cpos[j] = pos(lg.controls[j]);
  std::vector<Cd> E(size_t(D) * D, Cd(0, 0));
  for (int r = 0; r < D; r++)
    for (int c = 0; c < D; c++) {
      bool on = true;
      for (int j = 0; j < lg.nc; j++) on = on && ((c >> cpos[j]) & 1);
      if (!on) {
        if (r == c) E[size_t(r) * D + c] = 1.0;
        continue;
      }
      if ((uint32_t(r ^ c)) & ~tm) continue;
      int lr = 0, lc = 0;
      for (int j = 0; j < lg.k; j++) {
        lr |= ((r >> tpos[j]) & 1) << j;
        lc |= ((c >> tpos[j]) & 1) << j;
      }
      E[size_t(r) * D + c] = Cd(lg.m[lr][lc][0], lg.m[lr][lc][1]);
    }
  return E;
}

// The matrix M of an operation on qubits Sold, widened to the group S.
std::vector<Cd> widen(const std::vector<Cd>& M, const int* Sold, int kold, const int* S, int k) {
  const int D = 1 << k, Dold = 1 << kold;
  int p[5];
  uint32_t om = 0;
  for (int j = 0; j < kold; j++) {
    for (int t = 0; t < k; t++)
      if (S[t] == Sold[j]) p[j] = t;
    om |= 1u << p[j];
  }
  std::vector<Cd> W(size_t(D) * D, Cd(0, 0));
  for (int r = 0; r < D; r++)
    for (int c = 0; c < D; c++) {
      if ((uint32_t(r ^ c)) & ~om) continue;
      int lr = 0, lc = 0;
      for (int j = 0; j < kold; j++) {
        lr |= ((r >> p[j]) & 1) << j;
        lc |= ((c >> p[j]) & 1) << j;
      }
      W[size_t(r) * D + c] = M[size_t(lr) * Dold + lc];
    }
  return W;
}

std::vector<Cd> matmul(const std::vector<Cd>& A, const std::vector<Cd>& B, int D) {
  std::vector<Cd> C(size_t(D) * D, Cd(0, 0));
  for (int i = 0; i < D; i++)
    for (int m = 0; m < D; m++) {
      const Cd a = A[size_t(i) * D + m];
      if (a == Cd(0, 0)) continue;
      for (int j = 0; j < D; j++) C[size_t(i) * D + j] += a * B[size_t(m) * D + j];
    }
  return C;
}

int gate_qubit_list(const LocalGate& lg, int* q) {
  int u = 0;
  for (int j = 0; j < lg.k; j++) q[u++] = lg.targets[j];
  for (int j = 0; j < lg.nc; j++) q[u++] = lg.controls[j];
  return u;
}

bool diagonal_gate(const LocalGate& lg) {
  for (int r = 0; r < (1 << lg.k); r++)
    for (int c = 0; c < (1 << lg.k); c++)
      if (r != c && lg.structural[r][c]) return false;
  return true;
}

// Row factor of a diagonal gate on at most three qubits (targets, then
// controls): its diagonal on those qubits.
bool make_factor(const LocalGate& lg, DiagFactor* f) {
  int q[6];
  const int u = gate_qubit_list(lg, q);
  if (u > 3 || !diagonal_gate(lg)) return false;
  const std::vector<Cd> E = embed_gate(lg, q, u);
  std::memset(f, 0, sizeof(*f));
  f->k = u;
  for (int j = 0; j < u; j++) f->q[j] = q[j];
  for (int r = 0; r < (1 << u); r++) {
    f->v[r][0] = E[size_t(r) * (1 << u) + r].real();
    f->v[r][1] = E[size_t(r) * (1 << u) + r].imag();
  }
  return true;
}

struct BigArgs {
  int64_t ncos;
  int32_t nt;
  int32_t pad;
  int32_t sorted[5];
  int32_t pad2;
  int64_t off[32];  // global offset of local index r
  const double* mat;             // D x D, row-major, interleaved complex
  const char* tabs;              // factor tables applied to the output rows
};

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

template <typename R, int K>
__global__ __launch_bounds__(kBigBlock) void kron_big_kernel(BigArgs a, typename Vec<R>::V* __restrict__ v) {
  using V = typename Vec<R>::V;
  constexpr int D = 1 << K;
  __shared__ double2 sm[D * D];
  for (int t = threadIdx.x; t < D * D; t += kBigBlock) sm[t] = double2{a.mat[2 * t], a.mat[2 * t + 1]};
  __syncthreads();
  const int64_t c = int64_t(blockIdx.x) * kBigBlock + threadIdx.x;
  if (c >= a.ncos) return;
  int64_t base = c;
#pragma unroll
  for (int j = 0; j < K; j++) {
    const int p = a.sorted[j];
    base = (base & ((int64_t(1) << p) - 1)) | ((base >> p) << (p + 1));
  }
  double xr[D], xi[D];
#pragma unroll
  for (int r = 0; r < D; r++) {
    const V t = v[base + a.off[r]];
    xr[r] = double(t.x);
    xi[r] = double(t.y);
  }
  // each output row is written as soon as it is formed: the inputs stay in
  // registers, so the in-place update is safe
#pragma unroll
  for (int r = 0; r < D; r++) {
    // four independent partial sums per component keep the FMA chains short
    double pr[4] = {0, 0, 0, 0}, pi[4] = {0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < D; q++) {
      const double2 m = sm[r * D + q];
      pr[q & 3] = fma(m.x, xr[q], fma(-m.y, xi[q], pr[q & 3]));
      pi[q & 3] = fma(m.x, xi[q], fma(m.y, xr[q], pi[q & 3]));
    }
    double yr = (pr[0] + pr[1]) + (pr[2] + pr[3]);
    double yi = (pi[0] + pi[1]) + (pi[2] + pi[3]);
    const int64_t i = base + a.off[r];
    if (a.nt) apply_tables(a.tabs, a.nt, uint64_t(i), yr, yi);
    v[i] = V{R(yr), R(yi)};
  }
}

}  // namespace

diaq_status_t plan_big(const diaq_gate_t* gates, int64_t ngates, int n, int kmax, std::vector<BigOp>* ops) {
  if (kmax < 1 || kmax > 5) return fail(DIAQ_ERR_INVALID_ARGUMENT, "max_fused_qubits must be 1..5");
  ops->clear();
  for (int64_t gi = 0; gi < ngates; gi++) {
    LocalGate lg;
    diaq_status_t st = local_gate(&gates[gi], n, &lg);
    if (st != DIAQ_OK) return fail(st, "gate %lld: %s", (long long)gi, diaq_last_error());
    int gq[6];
    const int gu = gate_qubit_list(lg, gq);
    uint64_t gm = 0;
    for (int j = 0; j < gu; j++) gm |= uint64_t(1) << gq[j];
    int64_t host = -1;
    for (int64_t k = int64_t(ops->size()) - 1; k >= 0; k--)
      if ((*ops)[k].mask & gm) {
        host = k;
        break;
      }
    DiagFactor f;
    const bool is_diag = make_factor(lg, &f);
    if (host >= 0) {
      BigOp& X = (*ops)[host];
      uint64_t fm = 0;
      for (const auto& pf : X.post)
        for (int j = 0; j < pf.k; j++) fm |= uint64_t(1) << pf.q[j];
      int S[8];
      int k = X.k;
      for (int j = 0; j < k; j++) S[j] = X.q[j];
      for (int j = 0; j < gu; j++) {
        bool seen = false;
        for (int t = 0; t < k; t++) seen = seen || S[t] == gq[j];
        if (!seen && k < 8) S[k++] = gq[j];
      }
      if (!X.raw && k <= kmax && (is_diag || !(fm & gm))) {
        std::sort(S, S + k);
        const std::vector<Cd> A = widen(X.m, X.q, X.k, S, k);
        const std::vector<Cd> B = embed_gate(lg, S, k);
        X.m = matmul(B, A, 1 << k);  // g after the operation
        X.k = k;
        for (int j = 0; j < k; j++) X.q[j] = S[j];
        X.mask |= gm;
        X.ngates++;
        continue;
      }
      if (is_diag && int(X.post.size()) < kBigMaxFactors) {
        X.post.push_back(f);
        X.mask |= gm;  // later gates on these qubits must not move before it
        X.ngates++;
        continue;
      }
    } else if (is_diag && !ops->empty() && int(ops->back().post.size()) < kBigMaxFactors) {
      ops->back().post.push_back(f);
      ops->back().mask |= gm;
      ops->back().ngates++;
      continue;
    }
    BigOp op;
    op.mask = gm;
    op.ngates = 1;
    if (gu > 5) {
      // more than five qubits with its controls: applied as it is
      op.raw = true;
      op.lg = lg;
      op.k = gu;
    } else {
      op.k = gu;
      for (int j = 0; j < gu; j++) op.q[j] = gq[j];
      std::sort(op.q, op.q + gu);
      op.m = embed_gate(lg, op.q, gu);
    }
    ops->push_back(std::move(op));
  }
  return DIAQ_OK;
}

diaq_status_t run_big(diaq_ctx* ctx, const std::vector<BigOp>& ops, int n, diaq_dtype_t dt, void* state) {
  const int64_t N = int64_t(1) << n;
  // one table: every operation's matrix (2 D^2 doubles), then the factors
  std::vector<double> mats;
  std::vector<size_t> moff(ops.size());
  OpTables tabs;
  for (size_t k = 0; k < ops.size(); k++) {
    moff[k] = mats.size();
    for (const Cd& z : ops[k].m) {
      mats.push_back(z.real());
      mats.push_back(z.imag());
    }
    tabs.add(ops[k].post);
  }
  const size_t mb = ((mats.size() * sizeof(double) + 255) / 256) * 256;
  const size_t bytes = mb + tabs.bytes.size() + 256;
  DIAQ_TRY(ensure(ctx, &ctx->aux, bytes));
  char* base = static_cast<char*>(ctx->aux.ptr);
  DIAQ_TRY(upload(ctx, base, mats.data(), mats.size() * sizeof(double)));
  DIAQ_TRY(upload(ctx, base + mb, tabs.bytes.data(), tabs.bytes.size()));
  const double* dm = reinterpret_cast<const double*>(base);
  const double bytes_op = 2.0 * double(elem_bytes(dt)) * double(N);
  for (size_t k = 0; k < ops.size(); k++) {
    const BigOp& op = ops[k];
    const int nt = tabs.count[k];
    const char* tk = nt ? base + mb + tabs.first[k] : nullptr;
    const size_t e0 = prof_mark(ctx);
    if (op.raw) {
      DIAQ_TRY(launch_kron_apply(ctx, ctx->stream, op.lg, n, dt, state, false, tk, nt));
    } else if (op.k <= 3) {
      // small groups: the three-qubit kernels, controls already in the matrix
      LocalGate lg;
      std::memset(&lg, 0, sizeof(lg));
      lg.k = op.k;
      const int D = 1 << op.k;
      for (int j = 0; j < op.k; j++) {
        lg.targets[j] = op.q[j];
        lg.tmask |= uint64_t(1) << op.q[j];
      }
      for (int r = 0; r < D; r++)
        for (int c = 0; c < D; c++) {
          const Cd z = op.m[size_t(r) * D + c];
          lg.m[r][c][0] = z.real();
          lg.m[r][c][1] = z.imag();
          lg.structural[r][c] = z != Cd(0, 0);
        }
      DIAQ_TRY(launch_kron_apply(ctx, ctx->stream, lg, n, dt, state, false, tk, nt));
    } else {
      BigArgs a;
      std::memset(&a, 0, sizeof(a));
      a.ncos = N >> op.k;
      a.nt = nt;
      for (int j = 0; j < op.k; j++) a.sorted[j] = op.q[j];
      for (int r = 0; r < (1 << op.k); r++) {
        int64_t o = 0;
        for (int j = 0; j < op.k; j++)
          if ((r >> j) & 1) o |= int64_t(1) << op.q[j];
        a.off[r] = o;
      }
      a.mat = dm + moff[k];
      a.tabs = tk;
      const dim3 grid(unsigned((a.ncos + kBigBlock - 1) / kBigBlock)), block(kBigBlock);
      if (dt == DIAQ_C128) {
        if (op.k == 4) hipLaunchKernelGGL((kron_big_kernel<double, 4>), grid, block, 0, ctx->stream, a,
                                          static_cast<double2*>(state));
        else hipLaunchKernelGGL((kron_big_kernel<double, 5>), grid, block, 0, ctx->stream, a,
                                static_cast<double2*>(state));
      } else {
        if (op.k == 4) hipLaunchKernelGGL((kron_big_kernel<float, 4>), grid, block, 0, ctx->stream, a,
                                          static_cast<float2*>(state));
        else hipLaunchKernelGGL((kron_big_kernel<float, 5>), grid, block, 0, ctx->stream, a,
                                static_cast<float2*>(state));
      }
      DIAQ_HIP(hipGetLastError());
    }
    prof_interval(ctx, e0, prof_mark(ctx), 1, bytes_op);
  }
  return DIAQ_OK;
}

}  // namespace diaq

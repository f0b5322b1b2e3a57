// planner.cpp -- gate-level fusion for diaq_apply_circuit.
//
// Sec. VI fuses gates with the DiaQ matrix product before applying them.
// Fusing two expanded 2^n matrices costs O(d1 d2 N) and can multiply the
// diagonal count (GHZ(10) fused end to end has 1025 diagonals), so the
// product is taken on the gates' small local matrices instead (Alg. 1 on
// 2^k x 2^k DiaQ diagonals, k <= 3) and the fused gate is expanded once.
// A fusion is kept only if the fused gate moves no more HBM bytes than the
// gates applied one by one:  bytes(op) = s (2E + 2N)  (expansion writes E
// stored elements, the product reads them plus x and writes y).
// Diagonal gates that cannot join a core (too many qubits) are folded into
// the expansion as per-row phase factors, which leaves the diagonal set,
// hence the bytes, unchanged.
#include <complex>

#include "internal.hpp"

namespace diaq {

namespace {

using Cd = std::complex<double>;
constexpr int kMaxFactors = 64;

struct Local {
  int u = 0;       // number of qubits
  int q[3];        // q[0] = local least-significant bit
  Cd m[8][8];
};

int gate_qubits(const LocalGate& lg, int* out) {
  int c = 0;
  for (int j = 0; j < lg.k; j++) out[c++] = lg.targets[j];
  for (int j = 0; j < lg.nc; j++) out[c++] = lg.controls[j];
  return c;
}

uint64_t gate_mask(const LocalGate& lg) { return lg.tmask | lg.cmask; }

uint64_t op_mask(const FusedOp& op) {
  uint64_t m = gate_mask(op.core);
  for (const auto& f : op.post)
    for (int j = 0; j < f.k; j++) m |= uint64_t(1) << f.q[j];
  return m;
}

// Matrix of a gate over the ordered qubit list U: identity where a control
// is 0, the local matrix on the targets elsewhere.
void embed(const LocalGate& lg, const int* U, int u, Cd out[8][8]) {
  auto pos = [&](int qubit) {
    for (int j = 0; j < u; j++)
      if (U[j] == qubit) return j;
    return -1;
  };
  int tpos[3], cpos[3];
  uint32_t tm = 0;
  for (int j = 0; j < lg.k; j++) {
    tpos[j] = pos(lg.targets[j]);
    tm |= 1u << tpos[j];
  }
  for (int j = 0; j < lg.nc; j++) cpos[j] = pos(lg.controls[j]);
  const int d = 1 << u;
  for (int r = 0; r < d; r++)
    for (int c = 0; c < d; c++) {
      bool ctrl = true;
      for (int j = 0; j < lg.nc; j++) ctrl = ctrl && ((r >> cpos[j]) & 1);
      if (!ctrl) {
        out[r][c] = (r == c) ? Cd(1, 0) : Cd(0, 0);
        continue;
      }
      if ((uint32_t(r ^ c)) & ~tm) {
        out[r][c] = 0;
        continue;
      }
      int lr = 0, lc = 0;
      for (int j = 0; j < lg.k; j++) {
        lr |= ((r >> tpos[j]) & 1) << j;
        lc |= ((c >> tpos[j]) & 1) << j;
      }
      out[r][c] = Cd(lg.m[lr][lc][0], lg.m[lr][lc][1]);
    }
}

bool diag_nonzero(int d, const Cd M[8][8], int a) {
  for (int i = 0; i < d; i++) {
    const int j = i + a;
    if (j >= 0 && j < d && M[i][j] != Cd(0, 0)) return true;
  }
  return false;
}

// C = B * A by Alg. 1 on the local DiaQ diagonals: diagonal a of A and b of
// B add their element-wise product to diagonal a + b (summed, not assigned).
void local_product(int d, const Cd A[8][8], const Cd B[8][8], Cd C[8][8]) {
  for (int i = 0; i < d; i++)
    for (int j = 0; j < d; j++) C[i][j] = 0;
  for (int a = -(d - 1); a < d; a++) {
    if (!diag_nonzero(d, A, a)) continue;
    for (int b = -(d - 1); b < d; b++) {
      if (!diag_nonzero(d, B, b)) continue;
      const int c = a + b;
      if (c <= -d || c >= d) continue;
      for (int i = 0; i < d; i++) {
        const int m = i + b, j = i + c;
        if (m < 0 || m >= d || j < 0 || j >= d) continue;
        C[i][j] += B[i][m] * A[m][j];
      }
    }
  }
}

LocalGate to_local_gate(const int* U, int u, const Cd M[8][8]) {
  LocalGate lg;
  std::memset(&lg, 0, sizeof(lg));
  lg.k = u;
  lg.nc = 0;
  const int d = 1 << u;
  for (int j = 0; j < u; j++) {
    lg.targets[j] = U[j];
    lg.tmask |= uint64_t(1) << U[j];
  }
  for (int r = 0; r < d; r++)
    for (int c = 0; c < d; c++) {
      lg.m[r][c][0] = M[r][c].real();
      lg.m[r][c][1] = M[r][c].imag();
      lg.structural[r][c] = M[r][c] != Cd(0, 0);
    }
  return lg;
}

double op_bytes(const LocalGate& lg, int n, double s) {
  const double E = double(packing_starts(gate_offsets(lg), n).back());
  return s * (2.0 * E + 2.0 * double(int64_t(1) << n));
}

bool diagonal_factor(const diaq_gate_t* g, const LocalGate& lg, DiagFactor* f) {
  if (!is_diagonal_kind(g)) return false;
  int qs[6];
  const int u = gate_qubits(lg, qs);
  if (u > 3) return false;
  std::memset(f, 0, sizeof(*f));
  f->k = u;
  for (int j = 0; j < u; j++) f->q[j] = qs[j];
  Cd M[8][8];
  embed(lg, qs, u, M);
  for (int r = 0; r < (1 << u); r++) {
    f->v[r][0] = M[r][r].real();
    f->v[r][1] = M[r][r].imag();
  }
  return true;
}

}  // namespace

int compile_factors(const DiagFactor* f, int nf, std::vector<char>* out, const int64_t* off, int noff) {
  // group: each factor joins the table it widens least, within kTableQubits
  std::vector<uint64_t> gmask;
  std::vector<std::vector<int>> members;
  for (int j = 0; j < nf; j++) {
    uint64_t m = 0;
    for (int b = 0; b < f[j].k; b++) m |= uint64_t(1) << f[j].q[b];
    int best = -1, best_add = 65;
    for (size_t g = 0; g < gmask.size(); g++) {
      const int u = __builtin_popcountll(gmask[g] | m);
      if (u > kTableQubits) continue;
      const int add = u - __builtin_popcountll(gmask[g]);
      if (add < best_add) {
        best = int(g);
        best_add = add;
      }
    }
    if (best < 0) {
      gmask.push_back(0);
      members.emplace_back();
      best = int(gmask.size()) - 1;
    }
    gmask[best] |= m;
    members[best].push_back(j);
  }
  for (size_t g = 0; g < gmask.size(); g++) {
    int Q[64], nq = 0;
    for (int q = 0; q < 64; q++)
      if ((gmask[g] >> q) & 1) Q[nq++] = q;
    TableHead h;
    std::memset(&h, 0, sizeof(h));
    h.nq = nq;
    for (int i = 0; i < nq;) {
      int e = i;
      while (e + 1 < nq && Q[e + 1] == Q[e] + 1 && Q[e + 1] != 32) e++;
      h.run[h.nruns++] = Q[i] | ((e - i + 1) << 8) | (i << 16);
      i = e + 1;
    }
    for (int r = 0; r < noff && r < 32; r++)
      for (int j = 0; j < nq; j++)
        if ((uint64_t(off[r]) >> Q[j]) & 1) h.roff[r] = uint8_t(h.roff[r] | (1u << j));
    const size_t at = out->size();
    out->resize(at + table_bytes(nq));
    std::memcpy(out->data() + at, &h, sizeof(h));
    double* v = reinterpret_cast<double*>(out->data() + at + sizeof(h));
    // position of each factor qubit inside the table index
    for (int idx = 0; idx < (1 << nq); idx++) {
      Cd z(1, 0);
      for (int j : members[g]) {
        int r = 0;
        for (int b = 0; b < f[j].k; b++) {
          int pos = 0;
          while (Q[pos] != f[j].q[b]) pos++;
          r |= ((idx >> pos) & 1) << b;
        }
        z *= Cd(f[j].v[r][0], f[j].v[r][1]);
      }
      v[2 * idx] = z.real();
      v[2 * idx + 1] = z.imag();
    }
  }
  return int(gmask.size());
}

diaq_status_t plan_fusion(const diaq_gate_t* gates, int64_t ngates, int n, int kmax, diaq_dtype_t dt,
                          std::vector<FusedOp>* ops, bool kron) {
  if (kmax < 1 || kmax > 3) return fail(DIAQ_ERR_INVALID_ARGUMENT, "max_fused_qubits must be 1..3");
  const double s = double(elem_bytes(dt));
  ops->clear();
  for (int64_t gi = 0; gi < ngates; gi++) {
    LocalGate lg;
    diaq_status_t st = local_gate(&gates[gi], n, &lg);
    if (st != DIAQ_OK) return fail(st, "gate %lld: %s", (long long)gi, diaq_last_error());
    const uint64_t gm = gate_mask(lg);
    // latest op touching one of g's qubits: g commutes with every op after it
    int64_t host = -1;
    for (int64_t k = int64_t(ops->size()) - 1; k >= 0; k--)
      if (op_mask((*ops)[k]) & gm) {
        host = k;
        break;
      }
    DiagFactor f;
    const bool is_diag = diagonal_factor(&gates[gi], lg, &f);
    if (host >= 0) {
      FusedOp& X = (*ops)[host];
      // g may join the core only if it commutes with X's post factors
      uint64_t fm = 0;
      for (const auto& pf : X.post)
        for (int j = 0; j < pf.k; j++) fm |= uint64_t(1) << pf.q[j];
      int U[6];
      int u = gate_qubits(X.core, U);
      int gq[6];
      const int gu = gate_qubits(lg, gq);
      for (int j = 0; j < gu; j++) {
        bool seen = false;
        for (int t = 0; t < u; t++) seen = seen || U[t] == gq[j];
        if (!seen && u < 6) U[u++] = gq[j];
      }
      if (u <= kmax && (is_diag || !(fm & gm))) {
        Cd A[8][8], B[8][8], Cm[8][8];
        embed(X.core, U, u, A);
        embed(lg, U, u, B);
        local_product(1 << u, A, B, Cm);
        const LocalGate fused = to_local_gate(U, u, Cm);
        if (kron || op_bytes(fused, n, s) <= op_bytes(X.core, n, s) + op_bytes(lg, n, s)) {
          X.core = fused;
          X.ngates++;
          continue;
        }
      }
      if (is_diag && int(X.post.size()) < kMaxFactors) {
        X.post.push_back(f);
        X.ngates++;
        continue;
      }
    } else if (is_diag && !ops->empty() && int(ops->back().post.size()) < kMaxFactors) {
      // touches no earlier op: commutes with all of them
      ops->back().post.push_back(f);
      ops->back().ngates++;
      continue;
    }
    FusedOp op;
    op.core = lg;
    op.ngates = 1;
    ops->push_back(op);
  }
  return DIAQ_OK;
}

}  // namespace diaq

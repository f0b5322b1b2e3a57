// gates.cpp -- gate table and offset algebra of the time-step unitaries.
//
// A gate on targets t_0..t_{k-1} (t_0 = local bit 0) expands to the 2^n
// matrix I_above (x) Gate (x) I_below of Sec. II-C, generalised to
// non-adjacent and controlled qubits.  Its entry (i, j) can be non-zero only
// when i and j agree outside the targets, so j - i = scatter(c) - scatter(r)
// for local row r and column c; that set (plus 0 for a controlled gate,
// whose uncontrolled half is the identity) is its set of DiaQ diagonals
// (Sec. IV).  For adjacent targets this reduces to Alg. 3's
// dim_b * dIndex(M).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.hpp"

namespace diaq {

namespace {

struct C {
  double re, im;
};

C cexpi(double a) { return {std::cos(a), std::sin(a)}; }

int kind_targets(int kind) {
  switch (kind) {
    case DIAQ_GATE_SWAP:
    case DIAQ_GATE_RXX:
    case DIAQ_GATE_RYY:
    case DIAQ_GATE_RZZ:
      return 2;
    case DIAQ_GATE_MATRIX:
      return -1;  // any of 1..3
    default:
      return (kind >= DIAQ_GATE_I && kind <= DIAQ_GATE_U3) ? 1 : 0;
  }
}

void set(LocalGate* lg, int r, int c, C v) {
  lg->m[r][c][0] = v.re;
  lg->m[r][c][1] = v.im;
  lg->structural[r][c] = true;
}

// Pauli factors for the two-qubit rotations: <r|P|c> for P in {X, Y, Z}.
C pauli(int which, int r, int c) {
  if (which == 0) return (r != c) ? C{1, 0} : C{0, 0};              // X
  if (which == 1) {                                                  // Y
    if (r == c) return {0, 0};
    return (r == 0) ? C{0, -1} : C{0, 1};
  }
  return (r == c) ? C{r == 0 ? 1.0 : -1.0, 0} : C{0, 0};           // Z
}

C cmul(C a, C b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }

}  // namespace

bool is_diagonal_kind(const diaq_gate_t* g) {
  switch (g->kind) {
    case DIAQ_GATE_I: case DIAQ_GATE_Z: case DIAQ_GATE_S: case DIAQ_GATE_SDG:
    case DIAQ_GATE_T: case DIAQ_GATE_TDG: case DIAQ_GATE_RZ: case DIAQ_GATE_P:
    case DIAQ_GATE_RZZ:
      return true;
    default:
      return false;
  }
}

diaq_status_t local_gate(const diaq_gate_t* g, int n, LocalGate* lg) {
  if (!g) return fail(DIAQ_ERR_INVALID_ARGUMENT, "gate is NULL");
  if (n < 1 || n > 34) return fail(DIAQ_ERR_INVALID_ARGUMENT, "nqubits %d out of range [1, 34]", n);
  const int want = kind_targets(g->kind);
  if (want == 0) return fail(DIAQ_ERR_INVALID_ARGUMENT, "unknown gate kind %d", g->kind);
  if (g->ntargets < 1 || g->ntargets > 3 || (want > 0 && g->ntargets != want))
    return fail(DIAQ_ERR_INVALID_ARGUMENT, "gate kind %d takes %d targets, got %d", g->kind, want,
                g->ntargets);
  if (g->ncontrols < 0 || g->ncontrols > 3)
    return fail(DIAQ_ERR_INVALID_ARGUMENT, "ncontrols %d out of range [0, 3]", g->ncontrols);
  std::memset(lg, 0, sizeof(*lg));
  lg->k = g->ntargets;
  lg->nc = g->ncontrols;
  uint64_t seen = 0;
  for (int j = 0; j < lg->k + lg->nc; j++) {
    const int q = j < lg->k ? g->targets[j] : g->controls[j - lg->k];
    if (q < 0 || q >= n) return fail(DIAQ_ERR_INVALID_ARGUMENT, "qubit %d outside [0, %d)", q, n);
    if (seen & (1ull << q)) return fail(DIAQ_ERR_INVALID_ARGUMENT, "qubit %d used twice", q);
    seen |= 1ull << q;
    if (j < lg->k) {
      lg->targets[j] = q;
      lg->tmask |= 1ull << q;
    } else {
      lg->controls[j - lg->k] = q;
      lg->cmask |= 1ull << q;
    }
  }
  const double t = g->params[0];
  const double c = std::cos(0.5 * t), s = std::sin(0.5 * t);
  const double r2 = 1.0 / std::sqrt(2.0);
  switch (g->kind) {
    case DIAQ_GATE_I: set(lg, 0, 0, {1, 0}); set(lg, 1, 1, {1, 0}); break;
    case DIAQ_GATE_H:
      set(lg, 0, 0, {r2, 0}); set(lg, 0, 1, {r2, 0});
      set(lg, 1, 0, {r2, 0}); set(lg, 1, 1, {-r2, 0});
      break;
    case DIAQ_GATE_X: set(lg, 0, 1, {1, 0}); set(lg, 1, 0, {1, 0}); break;
    case DIAQ_GATE_Y: set(lg, 0, 1, {0, -1}); set(lg, 1, 0, {0, 1}); break;
    case DIAQ_GATE_Z: set(lg, 0, 0, {1, 0}); set(lg, 1, 1, {-1, 0}); break;
    case DIAQ_GATE_S: set(lg, 0, 0, {1, 0}); set(lg, 1, 1, {0, 1}); break;
    case DIAQ_GATE_SDG: set(lg, 0, 0, {1, 0}); set(lg, 1, 1, {0, -1}); break;
    case DIAQ_GATE_T: set(lg, 0, 0, {1, 0}); set(lg, 1, 1, cexpi(M_PI / 4)); break;
    case DIAQ_GATE_TDG: set(lg, 0, 0, {1, 0}); set(lg, 1, 1, cexpi(-M_PI / 4)); break;
    case DIAQ_GATE_SX:
      set(lg, 0, 0, {0.5, 0.5}); set(lg, 0, 1, {0.5, -0.5});
      set(lg, 1, 0, {0.5, -0.5}); set(lg, 1, 1, {0.5, 0.5});
      break;
    case DIAQ_GATE_RX:
      set(lg, 0, 0, {c, 0}); set(lg, 0, 1, {0, -s});
      set(lg, 1, 0, {0, -s}); set(lg, 1, 1, {c, 0});
      break;
    case DIAQ_GATE_RY:
      set(lg, 0, 0, {c, 0}); set(lg, 0, 1, {-s, 0});
      set(lg, 1, 0, {s, 0}); set(lg, 1, 1, {c, 0});
      break;
    case DIAQ_GATE_RZ: set(lg, 0, 0, cexpi(-0.5 * t)); set(lg, 1, 1, cexpi(0.5 * t)); break;
    case DIAQ_GATE_P: set(lg, 0, 0, {1, 0}); set(lg, 1, 1, cexpi(t)); break;
    case DIAQ_GATE_U3: {
      const double ph = g->params[1], la = g->params[2];
      const C el = cexpi(la), ep = cexpi(ph), epl = cexpi(ph + la);
      set(lg, 0, 0, {c, 0});
      set(lg, 0, 1, {-el.re * s, -el.im * s});
      set(lg, 1, 0, {ep.re * s, ep.im * s});
      set(lg, 1, 1, {epl.re * c, epl.im * c});
      break;
    }
    case DIAQ_GATE_SWAP:
      set(lg, 0, 0, {1, 0}); set(lg, 1, 2, {1, 0}); set(lg, 2, 1, {1, 0}); set(lg, 3, 3, {1, 0});
      break;
    case DIAQ_GATE_RXX:
    case DIAQ_GATE_RYY:
      // cos(t/2) I - i sin(t/2) P(x)P ; <r|P(x)P|c> = <r0|P|c0><r1|P|c1>
      for (int r = 0; r < 4; r++)
        for (int cc = 0; cc < 4; cc++) {
          const int which = g->kind == DIAQ_GATE_RXX ? 0 : 1;
          const C pp = cmul(pauli(which, r & 1, cc & 1), pauli(which, r >> 1, cc >> 1));
          C v = {pp.im * s, -pp.re * s};  // -i s * pp
          if (r == cc) v.re += c;
          if (r == cc || pp.re != 0.0 || pp.im != 0.0) set(lg, r, cc, v);
        }
      break;
    case DIAQ_GATE_RZZ:
      for (int r = 0; r < 4; r++) {
        const int parity = (r & 1) ^ (r >> 1);
        set(lg, r, r, cexpi(parity ? 0.5 * t : -0.5 * t));
      }
      break;
    case DIAQ_GATE_MATRIX: {
      if (!g->matrix) return fail(DIAQ_ERR_INVALID_ARGUMENT, "MATRIX gate without a matrix");
      const int d = 1 << lg->k;
      for (int r = 0; r < d; r++)
        for (int cc = 0; cc < d; cc++) {
          const double re = g->matrix[2 * (r * d + cc)], im = g->matrix[2 * (r * d + cc) + 1];
          if (re != 0.0 || im != 0.0) set(lg, r, cc, {re, im});
        }
      break;
    }
    default:
      return fail(DIAQ_ERR_INVALID_ARGUMENT, "unknown gate kind %d", g->kind);
  }
  return DIAQ_OK;
}

bool local_generator(const diaq_gate_t* g, LocalGate* lg) {
  // lg already holds the gate's qubits (from local_gate); replace the matrix.
  std::memset(lg->m, 0, sizeof(lg->m));
  std::memset(lg->structural, 0, sizeof(lg->structural));
  switch (g->kind) {
    case DIAQ_GATE_RX: set(lg, 0, 1, {1, 0}); set(lg, 1, 0, {1, 0}); return true;
    case DIAQ_GATE_RY: set(lg, 0, 1, {0, -1}); set(lg, 1, 0, {0, 1}); return true;
    case DIAQ_GATE_RZ: set(lg, 0, 0, {1, 0}); set(lg, 1, 1, {-1, 0}); return true;
    case DIAQ_GATE_P: set(lg, 1, 1, {-2, 0}); return true;
    case DIAQ_GATE_RXX:
    case DIAQ_GATE_RYY:
    case DIAQ_GATE_RZZ: {
      const int which = g->kind == DIAQ_GATE_RXX ? 0 : g->kind == DIAQ_GATE_RYY ? 1 : 2;
      for (int r = 0; r < 4; r++)
        for (int c = 0; c < 4; c++) {
          const C pp = cmul(pauli(which, r & 1, c & 1), pauli(which, r >> 1, c >> 1));
          if (pp.re != 0.0 || pp.im != 0.0) set(lg, r, c, pp);
        }
      return true;
    }
    default:
      return false;
  }
}

std::vector<int64_t> gate_offsets(const LocalGate& lg) {
  const int d = 1 << lg.k;
  int64_t sc[8];
  for (int r = 0; r < d; r++) {
    int64_t v = 0;
    for (int j = 0; j < lg.k; j++)
      if ((r >> j) & 1) v |= int64_t(1) << lg.targets[j];
    sc[r] = v;
  }
  std::vector<int64_t> offs;
  for (int r = 0; r < d; r++)
    for (int c = 0; c < d; c++)
      if (lg.structural[r][c]) offs.push_back(sc[c] - sc[r]);
  if (lg.nc > 0) offs.push_back(0);
  std::sort(offs.begin(), offs.end());
  offs.erase(std::unique(offs.begin(), offs.end()), offs.end());
  return offs;
}

std::vector<int64_t> packing_starts(const std::vector<int64_t>& offs, int n) {
  const int64_t N = int64_t(1) << n;
  std::vector<int64_t> st(offs.size() + 1, 0);
  for (size_t k = 0; k < offs.size(); k++) st[k + 1] = st[k] + (N - (offs[k] < 0 ? -offs[k] : offs[k]));
  return st;
}

uint64_t mask_from_offsets(const std::vector<int64_t>& offs) {
  // Smallest power of two >= |d| names the qubit a gate-shaped diagonal
  // couples (exact for +-2^q and +-(2^b - 2^a)); only a locality hint.
  uint64_t m = 0;
  for (int64_t d : offs) {
    uint64_t a = d < 0 ? uint64_t(-d) : uint64_t(d);
    if (!a) continue;
    int b = 63 - __builtin_clzll(a);
    if ((uint64_t(1) << b) != a) b++;
    if (b < 64) m |= uint64_t(1) << b;
  }
  return m;
}

}  // namespace diaq

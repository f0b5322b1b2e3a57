"""GPU parity of the Trotterised 1D TFIM workload (Hamiltonian simulation):
final states and the average magnetization under every plan, against the
CPU oracle."""
from __future__ import annotations

import pytest
import torch

from oracle import oracle as orc
from paper_2405_01250_amd import diaq as D
from paper_2405_01250_amd import inputs as W
from tests.gpu_util import assert_state_close, to_dev, to_host

pytestmark = pytest.mark.gpu

PLANS = {"plain": None, "dia+fuse2": dict(fuse=True, max_fused_qubits=2),
         "dia+fuse3": dict(fuse=True, max_fused_qubits=3), "kron": dict(kron=True),
         "kron+fuse3": dict(kron=True, fuse=True, max_fused_qubits=3)}


def _plan(name):
    kw = PLANS[name]
    return D.make_plan(**kw) if kw else None


@pytest.mark.parametrize("name", list(PLANS))
@pytest.mark.parametrize("n,steps", [(9, 6), (16, 4), (20, 3)])
def test_tfim_states_and_magnetization(n, steps, name):
    gates = W.tfim(n, steps, 0.1, J=1.0, hx=0.8)
    x = W.zero_state(n)
    ref = orc.apply_circuit(x, n, gates)
    psi = to_dev(x)
    D.apply_circuit(gates, psi, plan=_plan(name))
    assert_state_close(to_host(psi), ref, 1e-12, "TFIM n=%d %s" % (n, name))
    M = D.from_pauli_sum(n, W.magnetization_terms(n))
    m = D.expect(M, psi)
    want = orc.expect(n, W.magnetization_terms(n), ref)
    # |<M>| error <= 2 ||d psi|| ||M|| plus rounding of a 2^n-term sum
    assert abs(m - want) <= 1e-11


def test_tfim_energy_conserved_by_fine_steps():
    """exp(-i t H) conserves <H>; the Trotter circuit does so up to its
    step error, checked here on the GPU result from a random state."""
    n = 14
    x = W.random_state(n, 14)
    terms = W.tfim_terms(n)
    H = D.from_pauli_sum(n, terms)
    psi = to_dev(x)
    e0 = D.expect(H, psi).real
    D.apply_circuit(W.tfim(n, 200, 0.002), psi, plan=_plan("kron+fuse3"))
    e1 = D.expect(H, psi).real
    assert abs(e1 - orc.energy(x, n, W.tfim(n, 200, 0.002), terms)) <= 1e-11
    assert abs(e1 - e0) <= 5e-3


def test_tfim_complex64():
    n = 18
    gates = W.tfim(n, 4, 0.1)
    x = W.random_state(n, 18)
    ref = orc.apply_circuit(x, n, gates)
    for name in ("plain", "kron+fuse3"):
        psi = to_dev(x, torch.complex64)
        D.apply_circuit(gates, psi, plan=_plan(name))
        assert_state_close(to_host(psi), ref, 1e-5, "TFIM c64 %s" % name, l2tol=1e-4)


@pytest.mark.parametrize("name", ["plain", "kron+fuse3"])
def test_tfim_n28_full_state(name):
    """The benchmark's 28 spins and step, five Trotter steps (275 gates)
    compared on the whole state."""
    n = W.TFIM_N
    gates = W.tfim(n, 5, W.TFIM_DT)
    ref = orc.apply_circuit(W.zero_state(n), n, gates)
    psi = torch.zeros(1 << n, dtype=torch.complex128, device="cuda:0")
    psi[0] = 1
    D.apply_circuit(gates, psi, plan=_plan(name))
    M = D.from_pauli_sum(n, W.magnetization_terms(n))
    m = D.expect(M, psi).real
    got = to_host(psi)
    del psi, M
    torch.cuda.empty_cache()
    assert_state_close(got, ref, 1e-12, "TFIM n=28 %s" % name)
    assert abs(m - orc.expect(n, W.magnetization_terms(n), ref).real) <= 1e-11

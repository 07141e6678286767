"""CPU checks of the host factorisation the Newton loop starts from (cs_factor_host):
P and Q are permutations, T = (L - I) + U reproduces P A Q = L U on the oracle's
matrices (DC and backward-Euler stamps, voltage sources with their zero
diagonals, series resistors) without element growth, each source's node column
pivots on its branch row, the order keeps the fill of the 100,000-stage chain's
backward-Euler matrix linear, and a singular matrix is refused."""
import numpy as np
import pytest
import scipy.sparse as sp

from paper_2604_03079_amd import colorstamp as CS
from paper_2604_03079_amd import netgen as G

NC, PC = G.default_card(1), G.default_card(-1)


def factors(c, n, Ah):
    P, Q, Tp, Ti, Tx = c.factor_host(Ah)
    assert sorted(P.tolist()) == list(range(n)) and sorted(Q.tolist()) == list(range(n))
    T = sp.csr_matrix((Tx, Ti, Tp), shape=(n, n))
    assert np.all(np.diff(Ti[Tp[0]:Tp[1]]) > 0) if n > 1 and Tp[1] - Tp[0] > 1 else True
    L = sp.tril(T, -1) + sp.identity(n)
    U = sp.triu(T)
    return P, Q, L, U, T


CASES = [("chain50dc", lambda: G.chain_dc_case(50, 3), 0.0),
         ("chain50be", lambda: G.chain_dc_case(50, 3), 1e12),
         ("adder2r89", lambda: G.draw_params(G.split_nets(G.drive(G.drive(G.drive(
             G.ripple_adder28(2), 2, 1.0), 3, 0.0), 4, 1.0), "all")[0], np.random.default_rng(1),
             G.W_CHAIN, G.L_CHAIN), 1e12),
         ("opamp12", lambda: G.draw_params(G.opamp2(12), np.random.default_rng(2), G.W_OPAMP, G.L_OPAMP), 1e12),
         ("sram6x5", lambda: G.sram_case(6, 5, 8), 1e12),
         ("random300x40", lambda: G.with_random_resistors(G.draw_params(G.random_netlist(300, 40, 5),
                                                                         np.random.default_rng(3), G.W_CHAIN,
                                                                         G.L_CHAIN), 60, 4), 1e12)]


@pytest.mark.parametrize("name,make,ag0", CASES, ids=[c[0] for c in CASES])
def test_factors_reproduce_the_permuted_matrix(orc, name, make, ag0):
    circ = make()
    c = CS.prepare(circ, True)
    rp, ci = orc.pattern(circ)
    A, _ = orc.assemble(circ, rp, ci, NC, PC, ag0)
    n = circ.n_rows
    M = sp.csr_matrix((A, ci, rp), shape=(n, n))
    P, Q, L, U, T = factors(c, n, A)
    PAQ = M[P][:, Q]
    R = (L @ U - PAQ).toarray()
    assert np.abs(R).max() <= 1e-12 * abs(A).max()
    assert np.all(np.abs(U.diagonal()) > 0)
    if ag0 > 0:      # capacitive diagonals: no growth
        assert abs(T.data).max() <= 10 * abs(A).max()
    # sources first: the driven node's column pivots on the source's branch row
    nb = circ.n_nodes - 1
    for j, (p, q) in enumerate(circ.vsrc[:1]):
        assert Q[0] == p - 1 and P[0] == nb + j and Q[1] == nb + j and P[1] == p - 1


def test_fill_stays_linear_on_the_long_chain(orc):
    circ = G.chain_dc_case(100_000, 2)
    c = CS.prepare(circ, True)
    rp, ci = orc.pattern(circ)
    A, _ = orc.assemble(circ, rp, ci, NC, PC, 1e12)
    P, Q, Tp, Ti, Tx = c.factor_host(A)
    assert len(Ti) <= 2 * len(ci)
    assert abs(Tx).max() <= 10 * abs(A).max()


def test_singular_matrix_is_refused(orc):
    # at DC an undriven inverter input has a zero row and column: singular
    circ = G.workload(0)
    c = CS.prepare(circ, True)
    rp, ci = orc.pattern(circ)
    A, _ = orc.assemble(circ, rp, ci, NC, PC, 0.0)
    with pytest.raises(CS.CsError) as e:
        c.factor_host(A)
    assert e.value.status == -6


def _levels(n, Tp, Ti):
    lev = np.zeros(n, np.int64)
    for i in range(n):
        cols = Ti[Tp[i]:Tp[i + 1]]
        low = cols[cols < i]
        lev[i] = lev[low].max() + 1 if len(low) else 0
    return int(lev.max()) + 1


def test_order_choice_chain_and_split_adder(orc):
    # the chain keeps nested dissection (a shallow elimination, few dependency
    # levels); the adder with every net split takes minimum degree (far less fill
    # than the level-set separators of nested dissection give it)
    chain = G.chain_dc_case(20_000, 2)
    c = CS.prepare(chain, True)
    rp, ci = orc.pattern(chain)
    A, _ = orc.assemble(chain, rp, ci, NC, PC, 1e12)
    _, _, Tp, Ti, _ = c.factor_host(A)
    assert _levels(chain.n_rows, Tp, Ti) <= 80 and len(Ti) <= 2 * len(ci)
    adder = G.adder_case(16, 9, "all")
    c = CS.prepare(adder, True)
    rp, ci = orc.pattern(adder)
    A, _ = orc.assemble(adder, rp, ci, NC, PC, 1e12)
    P, Q, Tp, Ti, Tx = c.factor_host(A)
    assert len(Ti) <= 2 * len(ci)
    n = adder.n_rows
    M = sp.csr_matrix((A, ci, rp), shape=(n, n))
    T = sp.csr_matrix((Tx, Ti, Tp), shape=(n, n))
    L = sp.tril(T, -1) + sp.identity(n)
    assert np.abs((L @ sp.triu(T) - M[P][:, Q]).toarray()).max() <= 1e-12 * abs(A).max()

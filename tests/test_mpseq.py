"""The mass-preconditioning splittings (host logic, no GPU): sizes, chiralities and the telescoping
structure of Eqs.(noMP), (old_MP), (old_MP_N), (new_MP), (new_MP_N).  Their determinants are pinned
against the oracle in test_oracle_pins.py."""
import pytest

from paper_1710_09621_amd import mpseq as S

m, M = 0.01, 1.0


@pytest.mark.parametrize("hs", [[0.1], [0.05, 0.3], [0.03, 0.1, 0.4]])
def test_sizes(hs):
    N = len(hs)
    assert len(S.actions("old", m, hs, M)) == 2 * N + 2
    assert len(S.actions("new", m, hs, M)) == N + 2
    assert len(S.actions("none", m, (), M)) == 2


def test_one_heavy_mass_matches_the_paper():
    mh = 0.1
    assert S.actions("none", m, (), M) == [(-1, m, m, M), (+1, m, M, M)]
    assert S.actions("old", m, [mh], M) == [(-1, m, m, mh), (+1, m, mh, mh), (-1, mh, mh, M), (+1, mh, M, M)]
    assert S.actions("new", m, [mh], M) == [(-1, m, m, mh), (+1, m, mh, M), (-1, M, mh, M)]


@pytest.mark.parametrize("kind,hs", [("old", [0.05, 0.3]), ("new", [0.05, 0.3]), ("new", [0.03, 0.1, 0.4])])
def test_telescoping(kind, hs):
    st = S.chain(kind, m, hs, M)
    assert st[0] == (m, m) and st[-1] == (M, M)
    for a, b in zip(st, st[1:]):
        assert (a[0] == b[0]) != (a[1] == b[1])  # exactly one slot changes
    chir = [a[0] for a in S.actions(kind, m, hs, M)]
    assert all(c1 != c2 for c1, c2 in zip(chir, chir[1:])) or kind == "old"  # new MP alternates


def test_new_cascade_slots():
    h1, h2 = 0.05, 0.3
    assert S.chain("new", m, [h1, h2], M) == [(m, m), (m, h1), (h2, h1), (h2, M), (M, M)]
    assert S.chain("old", m, [h1, h2], M) == [(m, m), (m, h1), (h1, h1), (h1, h2), (h2, h2), (h2, M), (M, M)]


def test_rejects_bad_input():
    with pytest.raises(ValueError):
        S.actions("new", m, [0.5, 0.1], M)
    with pytest.raises(ValueError):
        S.actions("none", m, [0.1], M)
    with pytest.raises(ValueError):
        S.ratio_action((0.1, 0.2), (0.3, 0.4))
    with pytest.raises(ValueError):
        S.actions("both", m, [], M)

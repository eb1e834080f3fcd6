"""Host logic of the HMC driver: the time-scale levels of the splittings' factors (Sec. III)."""
from paper_1710_09621_amd import hmc, mpseq


def test_levels_follow_sec3():
    # Sec. III: the last factor of each splitting on the finer fermion time scale k1, the others on k2
    lv = {k: [a[0] for a in hmc.levels(mpseq.actions(k, 0.01, [] if k == "none" else [0.1], 1.0))]
          for k in ("none", "old", "new")}
    assert lv == {"none": [2, 1], "old": [2, 2, 2, 1], "new": [2, 2, 1]}
    new = hmc.levels(mpseq.actions("new", 0.01, [0.1], 1.0))
    assert new[-1][1:] == (-1, 1.0, 0.1, 1.0)

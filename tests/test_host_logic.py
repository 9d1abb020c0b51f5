"""Host logic of the Python layer, checked on the CPU: the cell field tables
the multiscale workflow builds from macroscopic samples (Sec. 5: each
macroscopic step of dt is n_sub cell steps with A linear in between)."""
import numpy as np

from paper_1804_01404_amd import pipeline


def test_micro_table_interpolates_between_macroscopic_samples():
    rng = np.random.default_rng(5)
    a = rng.normal(size=9)
    for n_sub, axis in ((1, 0), (3, 1), (4, 2)):
        tab = pipeline.micro_table(a, n_sub, axis)
        assert tab.shape == ((a.size - 1) * n_sub + 1, 3)
        others = [d for d in range(3) if d != axis]
        assert np.all(tab[:, others] == 0.0)
        for s in range(a.size - 1):
            for u in range(n_sub):
                want = a[s] + (u / n_sub) * (a[s + 1] - a[s])
                assert tab[s * n_sub + u, axis] == want
        assert tab[-1, axis] == a[-1]
        # every macroscopic sample is hit exactly
        assert np.array_equal(tab[::n_sub, axis], a)

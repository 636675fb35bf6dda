"""The cost model reproduces Table md-scheme (Sec. 2), stored with its
citation in tests/golden/md_scheme_table.txt."""
import os

from paper_2405_01834_amd import model
from tests.conftest import ROOT

CLASSES = {"[11|11]": (1, 1, 1, 1), "[33|33]": (3, 3, 3, 3), "[66|66]": (6, 6, 6, 6)}


def _rows():
    for line in open(os.path.join(ROOT, "tests", "golden", "md_scheme_table.txt")):
        if line.startswith("#") or not line.strip():
            continue
        cls, step, ain, aout, nf = line.split()
        yield cls, step, int(ain), int(aout), int(nf)


def test_table_md_scheme():
    for cls, step, ain, aout, nf in _rows():
        a_in, a_out, n_f = model.md_scheme(*CLASSES[cls])[step]
        assert (a_in, a_out) == (ain, aout), (cls, step)
        if (cls, step) == ("[66|66]", "pq"):
            # printed 103,514; the table's own formula gives 207,025/2 = 103,512.5
            assert n_f == 103512.5 and nf == 103514
        else:
            assert n_f == nf, (cls, step, n_f, nf)


def test_top_degree_saving_quoted_for_dd():
    """Sec. 2: applying Eq. (E2-abab) on the fly saves ~43% for |dd]: 1 - Ñ(3)/Ñ(4)."""
    assert abs(1 - model.ntil(3) / model.ntil(4) - 0.43) < 0.005


def test_shared_memory_example_of_v1():
    """Sec. 3 (V1): a |gg] ket needs 120 x 9 x 9 x 8 bytes = 78 KB, i.e. Ñ(7) = 120 with the top degree removed."""
    assert model.ntil(7) == 120 and 120 * 9 * 9 * 8 == 77760  # printed as 78KB

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


def test_eri3_model_counts_top_degree_rows():
    """(ab|P) with a one-centre auxiliary side: only its T_P = (l_P+1)(l_P+2)/2
    top-degree Hermite rows enter.  Hand count for (pd|f), K_ab = 2, K_P = 1:
    L = 6, R_6 = 8*13*78/8 = 1014, Ñ(3) = 20, T_3 = 10, N_ab = 15, N_P = 7:
    aux first  2*(1014 + 2*20*10*7) + 2*2*15*20*7 = 2*3814 + 8400 = 16028;
    pair first 2*(1014 + 2*15*20*10) + 2*15*10*7 = 2*7014 + 2100 = 16128."""
    assert model.R_L(6) == 1014 and model.top_degree(3) == 10
    assert model.eri3_flops(1, 2, 3, 2, 1) == 16028
    assert model.eri3_flops_pair_first(1, 2, 3, 2, 1) == 16128
    # aux first never counts more ket rows than the 4-centre form with l_d = 0
    for lP in range(7):
        assert model.eri3_flops(3, 3, lP, 1, 1) <= model.eri4_flops(3, 3, lP, 0, 1, 1)

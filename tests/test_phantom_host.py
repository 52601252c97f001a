"""Host-side checks of the synthetic workloads (no GPU)."""
import numpy as np

from paper_2509_20012_amd import phantom as ph


def test_dose_only_problem_keeps_dose_terms_and_matrices():
    p = ph.water32()
    q = p.dose_only()
    dose_bits = ph.DOSE_LO | ph.DOSE_HI | ph.OBJ_DOSE
    assert np.all((q.kind & ~np.uint16(dose_bits)) == 0)
    assert np.array_equal(q.kind, p.kind & np.uint16(dose_bits))
    assert np.any(q.kind & ph.DOSE_HI) and np.any(q.kind & ph.OBJ_DOSE)
    assert not np.any(q.kind & (ph.LETD_HI | ph.CDL_LO | ph.CDL_HI | ph.OBJ_CDL))
    assert q.d_val is p.d_val and q.l_val is p.l_val and q.col_idx is p.col_idx
    assert q.name.endswith("dose_only") and q.meta["problem"] == "dose only"

"""Host-side helpers of bench.py: the algorithmic byte model and the
sweeps-to-target rule."""
import bench


def test_long_path_bytes_sum_to_the_phase_figure():
    """The three long-path passes are charged so that they add up to the
    word phase's 8 + 8M and the doc phase's 12 + 8M bytes per token."""
    for M in (1, 2, 3, 4):
        for ph, whole in (("word", 8 + 8 * M), ("doc", 12 + 8 * M)):
            parts = sum(bench.algorithmic_bytes_per_token(f"{ph}_long_{p}", M) for p in ("hist", "mh", "draw"))
            assert parts == whole
            for b in ("g16", "g32", "wave", "block", "wide"):
                assert bench.algorithmic_bytes_per_token(f"{ph}_{b}", M) == whole


def test_sweeps_to_target_stays_within_tolerance():
    """S* is the first sweep count of the grid from which the curve stays
    within the tolerance of the reference (a curve that dips back out does
    not count until it stays in)."""
    ref = -100.0
    grid = bench.SWEEP_GRID
    curve = {s: ref * (1 + 0.05 / s) for s in grid}          # gap 5% / s
    assert bench.sweeps_to(curve, ref, 0.01) == min(s for s in grid if 0.05 / s <= 0.01)
    bumpy = dict(curve)
    bumpy[6] = ref * 1.2                                     # leaves the band again at 6
    assert bench.sweeps_to(bumpy, ref, 0.01) == min(s for s in grid if s > 6 and 0.05 / s <= 0.01)
    assert bench.sweeps_to({s: ref * 2 for s in grid}, ref, 0.01) is None

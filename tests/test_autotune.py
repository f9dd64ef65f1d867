"""The autotuner's selection and cache (host logic, no GPU)."""
from paper_1412_4825_amd import autotune


def test_pick_takes_fastest_and_keeps_first_of_ties(tmp_path):
    calls = []

    def trial(w, k):
        calls.append((w, k))
        return {(1024, 2): 3.0, (1024, 4): 2.0, (4096, 2): 2.0, (4096, 4): 5.0}[(w, k)]

    best = autotune.pick(trial, windows=(1024, 4096), wpbs=(2, 4), reps=2)
    assert (best["window"], best["wpb"], best["seconds"]) == (1024, 4, 2.0)
    assert len(best["table"]) == 4 and len(calls) == 8
    p = str(tmp_path / "sub" / "tune.json")
    assert autotune.load(p, "gamma") is None
    autotune.store(p, "gamma", best)
    autotune.store(p, "lda", {"window": 4096, "wpb": 8, "seconds": 1.0})
    assert autotune.load(p, "gamma") == {"window": 1024, "wpb": 4, "seconds": 2.0}
    assert autotune.load(p, "lda")["wpb"] == 8


def test_pick_uses_best_of_repeats():
    seq = iter([5.0, 1.0, 4.0, 4.0])
    best = autotune.pick(lambda w, k: next(seq), windows=(512, 1024), wpbs=(1,), reps=2)
    assert best["window"] == 512 and best["seconds"] == 1.0

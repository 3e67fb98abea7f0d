"""Plan cache of the tuner (host logic only; the tuners themselves are GPU calls, stubbed here)."""
import json

from paper_1707_03974_amd import tuning
import synth


class FakeProblem:
    def __init__(self, n_sites, bonds, U, n_up, n_dn):
        self.n_sites, self.bonds, self.U, self.n_up, self.n_dn = n_sites, bonds, U, n_up, n_dn
        self.tuned = 0
        self.plans = []

    def tune(self, dtype, reps=5):
        self.tuned += 1
        best = {"down": 3, "up_cw": 64, "up": 1, "map": 3}
        return best, [dict(best, ms=1.5), {"down": 1, "up_cw": 32, "up": 1, "map": 1, "ms": 2.0}]

    def set_plan(self, dtype, *plan):
        self.plans.append((dtype, plan))


class FakeBatch:
    def __init__(self, problems):
        self.problems = problems
        self.tuned = 0
        self.plans = []

    def tune(self, dtype, reps=5):
        self.tuned += 1
        best = {"tile_elems": 2048, "block": 1024, "wgs_per_cu": 4, "order": 1}
        return best, [dict(best, ms=0.2)]

    def set_plan(self, *plan):
        self.plans.append(plan)


def _ring(n, t=1.0, U=4.0, fill=2):
    return FakeProblem(n, [synth.Bond(i, (i + 1) % n, t) for i in range(n)], U, fill, fill)


def test_keys_depend_on_lattice_fillings_and_precision_not_on_U():
    a, b = _ring(8, U=4.0), _ring(8, U=7.5)
    assert tuning.plan_key(a, "f32", "gfx950") == tuning.plan_key(b, "f32", "gfx950")
    assert tuning.plan_key(a, "f32", "gfx950") != tuning.plan_key(a, "f64", "gfx950")
    assert tuning.plan_key(a, "f32", "gfx950") != tuning.plan_key(_ring(8, t=0.5), "f32", "gfx950")
    assert tuning.plan_key(a, "f32", "gfx950") != tuning.plan_key(_ring(8, fill=3), "f32", "gfx950")
    assert tuning.plan_key(a, "f32", "gfx950") != tuning.plan_key(a, "f32", "gfx942")
    # tuples and Bond objects describe the same lattice
    c = FakeProblem(8, [(b_.i, b_.j, b_.t) for b_ in a.bonds], 1.0, 2, 2)
    assert tuning.plan_key(a, "f32", "gfx950") == tuning.plan_key(c, "f32", "gfx950")
    p, q = _ring(8), _ring(10)
    assert tuning.batch_key([p, q], "f32", "gfx950") == tuning.batch_key([_ring(8), _ring(10)], "f32", "gfx950")
    assert tuning.batch_key([p, q], "f32", "gfx950") != tuning.batch_key([q, p], "f32", "gfx950")   # order = offsets


def test_problem_plan_is_tuned_once_then_read_back(tmp_path):
    path = str(tmp_path / "plans.json")
    g = _ring(8)
    e1, trials = tuning.tuned_plan(g, "f32", path=path, arch="gfx950")
    assert g.tuned == 1 and trials and e1["ms"] == 1.5
    e2, trials2 = tuning.tuned_plan(g, "f32", path=path, arch="gfx950")
    assert g.tuned == 1 and trials2 is None and e2 == e1
    assert g.plans[-1] == ("f32", (3, 64, 1, 3))
    tuning.tuned_plan(g, "f32", path=path, arch="gfx950", retune=True)
    assert g.tuned == 2
    with open(path) as f:
        assert len(json.load(f)) == 1


def test_batch_plan_is_tuned_once_then_read_back(tmp_path):
    path = str(tmp_path / "plans.json")
    b = FakeBatch([_ring(8), _ring(10)])
    tuning.tuned_batch_plan(b, "f64", path=path, arch="gfx950")
    e, trials = tuning.tuned_batch_plan(b, "f64", path=path, arch="gfx950")
    assert b.tuned == 1 and trials is None and b.plans[-1] == (2048, 1024, 4, 1)
    # problem and batch entries live side by side in one file
    tuning.tuned_plan(_ring(8), "f64", path=path, arch="gfx950")
    with open(path) as f:
        assert len(json.load(f)) == 2


def test_corrupt_cache_is_ignored(tmp_path):
    path = tmp_path / "plans.json"
    path.write_text("{not json")
    g = _ring(8)
    tuning.tuned_plan(g, "f32", path=str(path), arch="gfx950")
    assert g.tuned == 1 and json.loads(path.read_text())

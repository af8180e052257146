"""Host logic of the autotuner (paper_0807_2387_amd.tune) with a stand-in solver: the
coordinate search keeps each family's fastest candidate and carries it into the next
family's candidates, the cache round-trips through $FEMNFFT_TUNE_CACHE, and the key holds
what sets the shapes."""
import pytest

pytestmark = pytest.mark.cpu


class FakeSolver:
    """Stage times as a known function of the shapes; records what was set."""

    class P:
        grid, n, m, p, precision = 8192, 6144, 5, 5, 1

    def __init__(self):
        self.params = self.P()
        self.cur = dict(spread_groups=1, near_fwd_bx=32, near_fwd_by=8, near_fwd_cap=1024, near_adj_bx=32,
                        near_adj_by=8, near_adj_cap=512, tile=32)
        self.prof = False

    def shapes(self):
        return dict(self.cur)

    def set_shapes(self, **kw):
        self.cur.update(kw)

    def set_profiling(self, on):
        self.prof = on

    def set_charges(self, q):
        pass

    def eval(self):
        pass

    def adjoint_H(self, V):
        pass

    def profile(self):
        c = self.cur
        spread = 1.0 + 0.1 * c["spread_groups"] + (0.05 if c["tile"] == 16 else 0.0)
        near = 3.0 + abs(c["near_fwd_cap"] - 768) / 1000 + (0.2 if c["near_fwd_bx"] != 64 else 0.0)
        a_near = 2.0 + abs(c["near_adj_cap"] - 384) / 1000 + (0.3 if c["near_adj_bx"] != 16 else 0.0)
        return {"spread": (spread, 1), "a_spread": (spread, 1), "fold": (0.1, 1), "gather": (0.5, 1),
                "a_fold": (0.1, 1), "a_gather": (0.3, 1), "near": (near, 1), "a_near": (a_near, 1)}

    def info(self):
        return dict(win_ext=(2943, 2943), n_tgt=16775729, n_src=16810019, near_cells=5, n_surf=31224)


def test_coordinate_search_finds_the_minimum(monkeypatch):
    import sys
    import types
    fake_torch = types.SimpleNamespace(cuda=types.SimpleNamespace(synchronize=lambda: None))
    monkeypatch.setitem(sys.modules, "torch", fake_torch)
    from paper_0807_2387_amd import tune
    S = FakeSolver()
    best, trace = tune.tune(S, None, None, reps=1)
    assert best["tile"] == 32 and best["spread_groups"] == 1
    assert (best["near_fwd_bx"], best["near_fwd_by"], best["near_fwd_cap"]) == (64, 4, 768)
    assert (best["near_adj_bx"], best["near_adj_by"], best["near_adj_cap"]) == (16, 16, 384)
    assert S.cur == best
    # the adjoint family was searched with the forward winner in place
    adj = [c for c, fam, _ in trace if fam == "a_near"]
    assert adj and all(c["near_fwd_bx"] == 64 and c["near_fwd_cap"] == 768 for c in adj)


def test_cache_round_trip_and_key(tmp_path, monkeypatch):
    from paper_0807_2387_amd import tune
    monkeypatch.setenv("FEMNFFT_TUNE_CACHE", str(tmp_path / "sub" / "t.json"))
    monkeypatch.setattr(tune, "arch", lambda: "gfx950")
    k = tune.key_of(FakeSolver())
    assert k.startswith("gfx950|G8192|n6144|m5|p5|fp32|rn5|") and k.endswith("|surf1")
    assert tune.lookup(k) is None or tune.lookup(k) == tune.lookup(k)
    tune.store(k, {"tile": 16}, {"trials": 3})
    assert tune.lookup(k) == {"tile": 16}


def test_batch_tuning_searches_each_distinct_key_once(tmp_path, monkeypatch):
    """apply_batch: members with one key share one search (then a cache hit), every member
    gets its key's shapes, and a second call searches nothing."""
    import sys
    import types
    import paper_0807_2387_amd as pkg
    from paper_0807_2387_amd import tune
    fake_torch = types.SimpleNamespace(cuda=types.SimpleNamespace(synchronize=lambda: None))
    monkeypatch.setitem(sys.modules, "torch", fake_torch)
    monkeypatch.setenv("FEMNFFT_TUNE_CACHE", str(tmp_path / "t.json"))
    monkeypatch.setattr(tune, "PACKAGED", str(tmp_path / "none.json"))
    monkeypatch.setattr(tune, "arch", lambda: "gfx950")

    class MemberSolver(FakeSolver):
        def __init__(self, grid, m, p, eps_I, eps_B, precision, n, eps_S):
            super().__init__()
            self.params = types.SimpleNamespace(grid=grid, n=n, m=m, p=p, precision=precision)
            self.nt = self.ns = 0

        def set_geometry(self, y, x, w, n_surf=0):
            self.nt, self.ns = len(y), len(x)

        def info(self):
            return dict(win_ext=(100, 100), n_tgt=self.nt, n_src=self.ns, near_cells=5, n_surf=0)

    monkeypatch.setattr(pkg, "Solver", MemberSolver)
    searches = []
    real_tune = tune.tune
    monkeypatch.setattr(tune, "tune", lambda S, q, V, **kw: (searches.append(S.params.grid), real_tune(S, q, V, **kw))[1])

    class FakeBatch:
        def __init__(self, grids):
            self.params = [types.SimpleNamespace(grid=g, m=5, p=5, eps_I=0.01, eps_B=1 / 32, precision=1, n=0,
                                                 eps_S=0.0) for g in grids]
            self.set = {}

        def set_shapes(self, i, **sh):
            self.set[i] = sh

    B = FakeBatch([1024, 1024, 2048, 1024])
    sizes = [(20000, 40000), (20000, 40000), (20000, 40000), (200000, 400000)]
    toff = [0]
    soff = [0]
    for nt, ns in sizes:
        toff.append(toff[-1] + nt)
        soff.append(soff[-1] + ns)
    Y, X = list(range(toff[-1])), list(range(soff[-1]))
    res = tune.apply_batch(B, toff, Y, soff, X, X, X, Y, reps=1)
    keys = [r[0] for r in res]
    assert len(set(keys)) == 3 and keys[0] == keys[1] != keys[3]
    assert sorted(searches) == [1024, 1024, 2048] and [r[2] for r in res] == [True, False, True, True]
    assert all(B.set[i] == res[i][1] for i in range(4))
    res2 = tune.apply_batch(B, toff, Y, soff, X, X, X, Y, reps=1)
    assert not any(r[2] for r in res2) and len(searches) == 3

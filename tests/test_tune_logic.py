"""The autotuner's search on the CPU: timing and kernel queries are faked,
the launch-configuration table is the real library's (host-only calls)."""
import json

from paper_1809_09851_amd import fdbb as F
from paper_1809_09851_amd import tune


def _fake(monkeypatch, spill_ppt4=True):
    monkeypatch.setattr(tune, "workload", lambda op, dim, dtype, n: (lambda: None))
    calls = []

    def fake_time(fn, reps=7, warmup=2):
        cfg = F.fdbb_get_launch_config(calls[-1][0], calls[-1][1], calls[-1][2])
        block, ppt, cap, nt = cfg
        return 1.0 + abs(block - 256) / 1000.0 + (0.5 if cap else 0.0) + (0.01 if nt else 0.0) + ppt / 100.0

    def fake_info(op, dim, dtype, ppt, nt=1):
        calls.append((op, dim, dtype))
        return (128, 64 if (spill_ppt4 and ppt == 4) else 0)

    monkeypatch.setattr(tune, "time_launch", fake_time)
    monkeypatch.setattr(F, "fdbb_kernel_info", fake_info)


def test_search_skips_invalid_and_spilling_configs(monkeypatch):
    _fake(monkeypatch)
    old = F.fdbb_get_launch_config("flux_jacobian", 3, F.F64)
    try:
        res = tune.search("flux_jacobian", 3, "f64", 1 << 20)
        cfgs = [c for _, c in res]
        assert all(c[0] <= 256 for c in cfgs)          # staged kernels: at most 256 threads
        assert all(c[1] != 4 for c in cfgs)            # spilling kernels skipped
        assert res[0][1] == (256, 1, 0, 0)             # fastest under the fake clock
        assert F.fdbb_get_launch_config("flux_jacobian", 3, F.F64) == (256, 1, 0, 0)
    finally:
        F.fdbb_set_launch_config("flux_jacobian", 3, F.F64, *old)


def test_table_round_trip(tmp_path, monkeypatch):
    p = tmp_path / "t.json"
    key = "gfx950/hiptest"
    p.write_text(json.dumps({key: {
        "flux/3/f64": {"block": 128, "ppt": 2, "grid_cap": 0, "nt": 0},
        "fused/3/f64": {"block": 1024, "ppt": 1, "grid_cap": 0, "nt": 0},   # invalid: ignored
    }}))
    old = F.fdbb_get_launch_config("flux", 3, F.F64)
    oldf = F.fdbb_get_launch_config("fused", 3, F.F64)
    try:
        assert tune.apply_table(str(p), key=key) == 1
        assert F.fdbb_get_launch_config("flux", 3, F.F64) == (128, 2, 0, 0)
        assert F.fdbb_get_launch_config("fused", 3, F.F64) == oldf
    finally:
        F.fdbb_set_launch_config("flux", 3, F.F64, *old)


def test_table_round_trip_small_entries(tmp_path):
    p = tmp_path / "t.json"
    key = "gfx950/hiptest"
    p.write_text(json.dumps({key: {
        "small/flux/1/f64": {"max_n": 1 << 21, "block": 64, "ppt": 1, "grid_cap": 0, "nt": 1},
        "small/fused/3/f64": {"max_n": 1 << 21, "block": 1024, "ppt": 1, "grid_cap": 0, "nt": 1},  # refused
        "small/flux/1": {"max_n": 1},                                                            # malformed
    }}))
    saved = F.fdbb_get_small_launch_config("flux", 1, F.F64)
    try:
        assert tune.apply_table(str(p), key=key) == 1
        assert F.fdbb_get_small_launch_config("flux", 1, F.F64) == (1 << 21, 64, 1, 0, 1)
        assert F.fdbb_get_small_launch_config("fused", 3, F.F64)[0] == 0
    finally:
        F.fdbb_set_small_launch_config("flux", 1, F.F64, *saved) if saved[0] else \
            F.fdbb_set_small_launch_config("flux", 1, F.F64, 0)


def test_table_installs_the_server_batch_entry(tmp_path):
    p = tmp_path / "t.json"
    key = "gfx950/hiptest"
    p.write_text(json.dumps({key: {"serve_batch/0/mix": {"block": 128, "ppt": 2, "grid_per_cu": 8, "nt": 1}}}))
    saved = F.fdbb_get_server_batch_config()
    try:
        assert tune.apply_table(str(p), key=key) == 1
        assert F.fdbb_get_server_batch_config() == (128, 2, 8, 1)
    finally:
        F.fdbb_set_server_batch_config(*saved)


def test_search_small_installs_only_a_clear_winner(monkeypatch):
    """The small class is stored only when its best shape beats the large
    configuration at that size by more than the margin."""
    monkeypatch.setattr(tune, "workload", lambda op, dim, dtype, n: (lambda: None))
    monkeypatch.setattr(F, "fdbb_kernel_info", lambda *a, **k: (128, 0))
    op, dim, dt = "eos", 1, F.F64
    large = F.fdbb_get_launch_config(op, dim, dt)

    def clock(win):
        def t(fns, launches=256, rounds=2):
            m, b, p, g, nt = F.fdbb_get_small_launch_config(op, dim, dt)
            cfg = (b, p, g, nt)
            return 1.0 - (win if (m and cfg == (512, 2, 0, 1)) else 0.0)
        return t
    try:
        monkeypatch.setattr(tune, "time_queued", clock(0.10))
        res, large_ms, max_n = tune.search_small(op, dim, "f64", 1 << 20)
        assert large_ms == 1.0 and max_n == 1 << 21 and res[0][1] == (512, 2, 0, 1)
        assert F.fdbb_get_small_launch_config(op, dim, dt) == (1 << 21, 512, 2, 0, 1)
        assert F.fdbb_launch_config_for(op, dim, dt, 1 << 20) == (512, 2, 0, 1)
        assert F.fdbb_launch_config_for(op, dim, dt, 1 << 22) == large
        monkeypatch.setattr(tune, "time_queued", clock(0.01))
        res, large_ms, max_n = tune.search_small(op, dim, "f64", 1 << 20)
        assert max_n == 0 and F.fdbb_get_small_launch_config(op, dim, dt)[0] == 0
    finally:
        F.fdbb_set_small_launch_config(op, dim, dt, 0)


def test_main_skips_an_op_with_no_usable_configuration(tmp_path, monkeypatch):
    """When every configuration spills (or is refused), the tuner reports it
    and writes no entry instead of failing."""
    monkeypatch.setattr(tune, "search", lambda *a, **k: [])
    monkeypatch.setattr(tune, "arch_key", lambda: "gfx950/hiptest")
    monkeypatch.setattr(tune.torch.cuda, "set_device", lambda d: None)
    out = tmp_path / "t.json"
    assert tune.main(["--ops", "adjoint", "--dims", "3", "--dtypes", "f64", "--n", "1024",
                      "--write", str(out)]) == 0
    assert json.loads(out.read_text()) == {"gfx950/hiptest": {}}

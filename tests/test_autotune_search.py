"""The autotuner's coordinate descent on synthetic cost models (host logic, no GPU)."""
from paper_2306_07872_amd import autotune

BASE = dict(t_lane=256, t_wave=2048, grid=0)


def test_noise_does_not_move_the_defaults():
    space = {"t_lane": [16, 64, 256, 1024], "t_wave": [256, 1024, 2048, 8192]}
    best, t = autotune.descend(space, BASE, 256, 1.0, lambda tr: 0.99, min_gain=0.03)
    assert best == {} and t <= 1.0


def test_clear_win_is_taken_and_rejected_combinations_are_skipped():
    def cost(tr):
        lane, wave = tr.get("t_lane", 256), tr.get("t_wave", 2048)
        if wave < lane:
            return None  # the library rejects t_wave below t_lane
        return {16: 2.0, 64: 1.5, 256: 1.0, 1024: 0.8}[lane] * (1.0 if wave >= 1024 else 1.2)

    seen = []

    def logged(tr):
        seen.append(dict(tr))
        return cost(tr)

    space = {"t_lane": [16, 64, 256, 1024], "t_wave": [256, 1024, 2048, 8192]}
    best, t = autotune.descend(space, BASE, 256, 1.0, logged)
    assert best["t_lane"] == 1024 and best.get("t_wave", 2048) >= 1024
    assert abs(t - 0.8) < 1e-12
    assert {"t_lane": 1024, "t_wave": 256} in seen  # tried, rejected, skipped


def test_every_candidate_rejected_leaves_the_field_alone():
    best, t = autotune.descend({"t_wave": [8, 16]}, BASE, 256, 1.0, lambda tr: None)
    assert best == {} and t == 1.0


def test_grid_per_compute_unit_starts_from_the_held_grid():
    base = dict(BASE, grid=512)
    seen = []

    def cost(tr):
        seen.append(tr.get("grid_per_cu"))
        return 0.5 if tr.get("grid_per_cu") == 4 else 1.0

    best, t = autotune.descend({"grid_per_cu": [1, 4]}, base, 256, 1.0, cost)
    assert 2 in seen  # 512 workgroups on 256 compute units, always a candidate
    assert best == {"grid_per_cu": 4} and t == 0.5
    assert autotune._to_tuning(best, 256)["grid"] == 1024

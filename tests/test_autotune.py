"""Host logic of the launch autotuner (no GPU): the committed table and the
lookup that maps a lattice side to (placement, walkers per wavefront)."""
import json
import os

from paper_1302_2320_amd import autotune


def test_committed_table_is_well_formed():
    table = autotune.load_table()
    assert table, "paper_1302_2320_amd/tune_table.json is missing"
    for L, e in table.items():
        assert L % 2 == 0 and 4 <= L <= 256
        assert e["wpw"] in (0, 16, 32, 64)
        # placements with state in LDS exist only for L <= 64
        assert e["placement"] in ((1, 2, 3, 5, 6, 7) if L <= 64 else (0, 1))
        best = max(e["candidates"], key=lambda c: c["attempts_per_s"])
        assert (best["placement"], best["wpw"]) == (e["placement"], e["wpw"])
        assert e.get("check_factor", 16) in autotune.CHECK_FACTORS
        done = [c for c in e.get("check_candidates", []) if c["seconds"] is not None]
        if done:
            assert min(done, key=lambda c: c["seconds"])["factor"] == e["check_factor"]


def test_choice_for_nearest_entry_same_side_of_64():
    table = {16: {"placement": 1, "wpw": 64}, 64: {"placement": 2, "wpw": 64},
             128: {"placement": 0, "wpw": 32}}
    assert autotune.choice_for(16, table) == (1, 64)
    assert autotune.choice_for(20, table) == (1, 64)
    assert autotune.choice_for(60, table) == (2, 64)
    # a lattice wider than 64 never takes an LDS placement tuned for L <= 64
    assert autotune.choice_for(66, table) == (0, 32)
    assert autotune.choice_for(256, table) == (0, 32)
    assert autotune.choice_for(32, {}) == (0, 0)


def test_representative_lines_cover_the_half_range():
    lines = autotune.representative_lines(16, 100)
    ells = sorted(p.ell for p in lines)
    assert len(lines) == 100 and ells[0] == 1 and ells[-1] == 16 * 16 // 2
    assert all(p.L == 16 for p in lines)


def test_load_table_missing_file(tmp_path):
    assert autotune.load_table(os.path.join(str(tmp_path), "none.json")) == {}


def test_check_factor_lookup():
    table = {16: {"placement": 1, "wpw": 64, "check_factor": 4}, 128: {"placement": 0, "wpw": 32}}
    assert autotune.check_factor_for(24, table) == 4
    assert autotune.check_factor_for(256, table) == autotune.DEFAULT_CHECK_FACTOR
    assert autotune.check_factor_for(8, {}) == autotune.DEFAULT_CHECK_FACTOR


def test_library_header_matches_the_table():
    """build.py compiles tune_table.json into csrc/wl_tune_table.h; the two agree."""
    path = os.path.join(os.path.dirname(autotune.TABLE), "csrc", "wl_tune_table.h")
    with open(path) as f:
        assert f.read() == autotune.c_header(autotune.load_table())

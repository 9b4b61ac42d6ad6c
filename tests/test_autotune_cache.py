"""Autotuner host logic: problem keys, candidate sets, cached lookups (no GPU)."""
import json

import workloads as wl
from paper_2608_25830_amd import autotune as AT


def test_keys_bucket_N_and_separate_groups():
    a = wl.make_workload("arm7", 0, N=1500)
    b = wl.make_workload("arm7", 0, N=2048)
    c = wl.make_workload("2d-large", 0, N=2048)
    assert AT.problem_key(a) == AT.problem_key(b)
    assert AT.problem_key(b) != AT.problem_key(c)
    assert AT.problem_key(b).startswith("arm7:K40:")
    # M scales the tile count as N does; the key names the library build
    d = wl.make_workload("arm7", 0, N=2048, M=4)
    assert AT.problem_key(d) != AT.problem_key(b)
    assert AT.problem_key(b).endswith(":lib" + AT.library_tag()) and len(AT.library_tag()) == 12


def test_entries_of_another_library_build_are_not_reused(tmp_path):
    w = wl.make_workload("2d-small", 0)
    path = tmp_path / "t.json"
    stale = AT.problem_key(w).rsplit(":lib", 1)[0] + ":lib000000000000"
    path.write_text(json.dumps({stale: dict(states_per_iter=2, sphere_chunks=0, blocks_per_cu=1, ms=0.5, table=[])}))
    AT._MEM.clear()
    assert AT.problem_key(w) not in json.loads(path.read_text())
    AT._MEM.clear()


def test_candidates_cover_each_knob():
    arm = AT.candidates(wl.make_workload("arm7", 0))
    pt = AT.candidates(wl.make_workload("2d-small", 0))
    assert {c["sphere_chunks"] for c in arm} == {0, 1, 2, 4}
    assert {c["states_per_iter"] for c in pt} == {0, 1, 2, 4, 8}
    assert {c["sphere_chunks"] for c in pt} == {0, 2}
    assert len({tuple(sorted(c.items())) for c in pt}) == len(pt)
    assert len({tuple(sorted(c.items())) for c in arm}) == len(arm)


def test_cached_entry_is_returned_without_timing(tmp_path):
    w = wl.make_workload("2d-small", 0)
    path = tmp_path / "t.json"
    entry = dict(states_per_iter=2, sphere_chunks=0, blocks_per_cu=1, ms=0.5, table=[])
    path.write_text(json.dumps({AT.problem_key(w): entry}))
    AT._MEM.clear()
    assert AT.tune_edge(w, cache_path=str(path)) == entry
    AT._MEM.clear()

"""Host-side pair schedule of the library (md_schedule_preview; no GPU needed).

The evaluation kernel adds each pair's force into its lane group's force copy without atomics,
which is only correct if no atom occurs twice within a group's part of a row.  These tests
check that invariant, and that the schedule holds exactly the oracle's intramolecular pair list
(built independently, in Python), for many ligands and plans."""
import numpy as np
import pytest

from oracle import ligand as OL
from workload import configs, synth

md = pytest.importorskip("paper_2203_02096_amd")

CASES = [(4, 1), (6, 2), (10, 3), (20, 4), (33, 7), (40, 8), (64, 12), (65, 12), (90, 20), (128, 32)]
PLANS = [dict(), dict(group_div=2), dict(group_div=4), dict(group_div=8, waves_per_block=1),
         dict(lds_budget=0), dict(lds_budget=160 * 1024, waves_per_block=8), dict(lds_budget=20000),
         dict(waves_per_block=4, waves_per_pose=4), dict(lds_budget=160 * 1024, waves_per_block=8, waves_per_pose=2),
         dict(group_div=8, waves_per_block=8), dict(lds_budget=160 * 1024, waves_per_block=16),
         dict(lds_budget=160 * 1024, waves_per_block=12, group_div=2)]


def _lib_available():
    try:
        md.lib()
        return True
    except Exception:
        return False


pytestmark = pytest.mark.skipif(not _lib_available(), reason="libmdock.so not built")


@pytest.mark.parametrize("n,t", CASES)
@pytest.mark.parametrize("plan", range(len(PLANS)))
def test_schedule_invariants(n, t, plan):
    lig = synth.make_ligand(n, t, 5000 + 7 * n + t, configs.type_params())
    info, slots, m = md.md_schedule_preview(lig, **PLANS[plan])
    ol = OL.from_synth(lig)
    rows = info["total_rows"]
    assert slots.size == rows * 64
    empty = (slots >> 17) & 1
    i = slots & 0xFF
    j = (slots >> 8) & 0xFF
    # empty slots name atom N at both ends; real slots hold the oracle's pairs, each exactly once
    assert np.all(i[empty == 1] == n) and np.all(j[empty == 1] == n)
    real = np.stack([i[empty == 0], j[empty == 0]], 1)
    assert real.shape[0] == len(ol.pairs)
    # a slot may hold its pair either way round (the kernel's pair term is symmetric)
    assert np.all(real[:, 0] != real[:, 1]) and np.all(real < n)
    real = np.sort(real, axis=1)
    got = sorted(map(tuple, real.tolist()))
    want = sorted(map(tuple, np.asarray(ol.pairs).reshape(-1, 2).tolist()))
    assert got == want
    # no atom twice within a lane group's part of a row
    assert 1 <= m <= 64
    for r in range(rows):
        for g0 in range(0, 64, m):
            seg = slice(r * 64 + g0, r * 64 + min(64, g0 + m))
            atoms = np.concatenate([i[seg][empty[seg] == 0], j[seg][empty[seg] == 0]])
            assert len(np.unique(atoms)) == len(atoms), (r, g0)
    # the H-bond pairs sit in the first rows (the rows after them need no per-slot choice of the
    # 12-10 form); the H-bond-free rows are at least the rows beyond the ones the H-bond pairs
    # need on their own, unless that layout took more rows than one mixed sequence
    hb = (slots >> 16) & 1
    has_hb = [bool(np.any(hb[r * 64:(r + 1) * 64][empty[r * 64:(r + 1) * 64] == 0])) for r in range(rows)]
    last = max([r + 1 for r in range(rows) if has_hb[r]], default=0)
    assert all(has_hb[:last]) or rows * 64 <= 1.2 * len(ol.pairs) + 128
    # close to the minimum number of rows (one more for the separate H-bond rows)
    assert rows >= -(-len(ol.pairs) // 64)
    assert rows * 64 <= 1.2 * len(ol.pairs) + 192
    # LDS: staged rows within the budget, and as many as fit; the pair loop's prefetch reads one
    # row behind the staged ones, which is staged too
    budget = PLANS[plan].get("lds_budget", 65536)
    assert info["lds_bytes"] <= 160 * 1024
    assert 0 <= info["staged_rows"] <= rows
    per_row = 64 * 20
    staged = info["staged_rows"] + (1 if info["staged_rows"] > 0 else 0)
    fixed = info["lds_bytes"] - staged * per_row
    assert fixed > 0
    if info["staged_rows"] > 0:
        assert info["lds_bytes"] <= budget
    if info["staged_rows"] < rows:
        assert info["lds_bytes"] + (per_row if info["staged_rows"] > 0 else 2 * per_row) > budget


def test_schedule_preview_rejects_bad_plans():
    lig = synth.make_ligand(20, 4, 77, configs.type_params())
    for bad in (dict(group_div=1), dict(group_div=9), dict(waves_per_block=3), dict(waves_per_block=32),
                dict(waves_per_block=10), dict(lds_budget=-1),
                dict(lds_budget=160 * 1024 + 1), dict(waves_per_pose=3), dict(waves_per_pose=8)):
        with pytest.raises(md.MdockError):
            md.md_schedule_preview(lig, **bad)


@pytest.mark.parametrize("n,t", [(20, 4), (65, 12), (128, 32)])
@pytest.mark.parametrize("wpp", [2, 4])
def test_shared_pose_layout(n, t, wpp):
    """A plan whose waves share a pose holds one pose per block (waves_per_block = waves_per_pose)
    and adds to the W waves' own LDS exactly the shared arrays the kernel addresses: the pose's
    coordinates 3 x 4 x (64A + 1) (rounded up to 16 bytes), its torsion gradients 4 x 64 and two
    share sets 2 x 16 x ((W + 1)(N + 1) + W) bytes."""
    lig = synth.make_ligand(n, t, 6000 + n, configs.type_params())
    shared, s1, _ = md.md_schedule_preview(lig, lds_budget=0, waves_per_block=8, waves_per_pose=wpp)
    alone, s2, _ = md.md_schedule_preview(lig, lds_budget=0, waves_per_block=wpp)
    assert shared["waves_per_block"] == wpp and shared["waves_per_pose"] == wpp
    assert alone["waves_per_pose"] == 1
    assert np.array_equal(s1, s2)                       # the pair schedule itself is unchanged
    assert shared["staged_rows"] == alone["staged_rows"] == 0
    A = 2 if n > 64 else 1
    coords = -(-12 * (64 * A + 1) // 16) * 16
    assert shared["lds_bytes"] - alone["lds_bytes"] == coords + 4 * 64 + 2 * 16 * ((wpp + 1) * (n + 1) + wpp)



_PREVIEW_SCRIPT = """
import hashlib, sys
sys.path.insert(0, sys.argv[1])
import paper_2203_02096_amd as md
from workload import configs, synth
for n, t in ((20, 4), (65, 12), (128, 32)):
    info, slots, m = md.md_schedule_preview(synth.make_ligand(n, t, 9000 + n, configs.type_params()))
    print(n, sorted(info.items()), m, hashlib.sha256(slots.tobytes()).hexdigest())
"""


def _preview_digest(lig, **plan):
    info, slots, m = md.md_schedule_preview(lig, **plan)
    return sorted(info.items()), m, slots.tobytes()


@pytest.mark.parametrize("n,t", [(20, 4), (65, 12), (128, 32)])
def test_two_creations_give_the_same_schedule(n, t):
    """The schedule is a function of the ligand alone: two creations from separate copies of the
    same arrays, and one after planning other ligands in between, give the same plan and the
    same slots byte for byte."""
    tp = configs.type_params()
    first = _preview_digest(synth.make_ligand(n, t, 9000 + n, tp))
    for k in range(3):
        md.md_schedule_preview(synth.make_ligand(10 + 17 * k, 2 + k, 31 + k, tp), group_div=2 + k)
    again = synth.make_ligand(n, t, 9000 + n, tp)
    copy = synth.Ligand(again.xyz.copy(), again.types.copy(), again.charges.copy(), again.bonds.copy(),
                        again.torsions.copy(), again.root, again.type_params.copy())
    assert _preview_digest(copy) == first


def test_schedule_same_in_a_fresh_process():
    """Nothing in the planner depends on addresses or on process state: a second process plans
    the same ligands to the same slots."""
    import hashlib
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    outs = [subprocess.run([sys.executable, "-c", _PREVIEW_SCRIPT, root], capture_output=True, text=True,
                           timeout=120, check=True).stdout for _ in range(2)]
    assert outs[0] == outs[1] and len(outs[0].splitlines()) == 3
    here = []
    for n, t in ((20, 4), (65, 12), (128, 32)):
        info, m, raw = _preview_digest(synth.make_ligand(n, t, 9000 + n, configs.type_params()))
        here.append(f"{n} {info} {m} {hashlib.sha256(raw).hexdigest()}")
    assert outs[0].splitlines() == here


@pytest.mark.parametrize("n,t", [(20, 4), (64, 12), (65, 12), (128, 32)])
def test_widest_blocks(n, t):
    """16 waves per block for one atom per lane; two atoms per lane (more than 64 atoms) take at
    most 12 (three waves per SIMD), so a request for 16 is reduced to 12."""
    lig = synth.make_ligand(n, t, 7000 + n, configs.type_params())
    info, _, _ = md.md_schedule_preview(lig, lds_budget=160 * 1024, waves_per_block=16)
    assert info["waves_per_block"] == (16 if n <= 64 else 12)
    assert info["lds_bytes"] <= 160 * 1024


def _bank_cycles_per_row(slots, m, n_atoms):
    """LDS cycles one row's pair loop spends, per a model of the LDS: 32 four-byte banks serving 32
    lanes at a time, each access taking as many cycles as its busiest bank has distinct words.
    Per half-row and atom side: the x-y pair and z of the coordinates (pitch 64A + 1 words) and of
    the lane group's force copy (read and written, so twice)."""
    A = 2 if n_atoms > 64 else 1
    pitch = 64 * A + 1
    copy = ((12 * pitch + 15) // 16 * 16) // 4
    group = np.arange(64) // m
    rows = slots.reshape(-1, 64)
    total = 0
    for row in rows:
        for atoms in (row & 0xFF, (row >> 8) & 0xFF):
            for h in (slice(0, 32), slice(32, 64)):
                a, g = atoms[h].astype(np.int64), group[h]
                for base, weight in ((a, 1), (a + g * copy, 2)):
                    for words in (np.concatenate([base, base + pitch]), base + 2 * pitch):
                        w = np.unique(words)
                        total += weight * np.bincount(w % 32, minlength=32).max()
    return total / len(rows)


# (atoms, torsions, seed, modelled cycles per row of a first-fit placement of the same pairs:
# each pair, in the same priority order, into the first group where both its atoms are free)
BANK_CASES = [(73, 14, 11, 72.1), (87, 17, 12, 78.5), (90, 20, 13, 79.4), (120, 24, 14, 86.3)]


@pytest.mark.parametrize("n,t,seed,first_fit", BANK_CASES)
def test_pair_rows_spread_over_lds_banks(n, t, seed, first_fit):
    """The row builder places each pair in the group and orientation that add the fewest LDS
    bank-conflict cycles (ideal: 36 per row).  For ligands of two atoms per lane it keeps the
    modelled cycles per row at least 10 % below a first-fit placement's."""
    lig = synth.make_ligand(n, t, 9100 + seed, configs.type_params())
    info, slots, m = md.md_schedule_preview(lig, group_div=2)
    assert m == 32
    assert _bank_cycles_per_row(slots, m, n) < 0.9 * first_fit

"""The index plan of the record's wave-cooperative tape writes, checked on the
CPU (no GPU): for every record size the explicit pairs can have and any set
of lanes completing a group, the rounds write every chunk of every completed
group exactly once, to its place in the group, from that lane's LDS slot,
and every LDS and queue index stays inside its array.  The plan restated
here is the one the kernel follows (flush_groups_wave, wave_flush_parts,
stage_rec_sw in the record's source): lanes ranked among the live ones,
G chunks a group, `per` = live // G groups a round, chunk c of lane l
staged at c * 256 + (l xor (c mod 8)).
"""
import numpy as np
import pytest

TAPE_GROUP = 4


def record_chunks(d, elem_bytes):
    """16-byte chunks of one tape record: the step size, then the state,
    padded to 16 bytes."""
    return ((8 + d * elem_bytes) + 15) // 16


def stage_index(c, tid):
    return c * 256 + (tid ^ (c & 7))


def plan(live_mask, need_mask, wave, g):
    """Writes [(group owner lane, chunk, LDS index read, queue index read)]
    of one call, following the kernel's rounds."""
    live = [l for l in range(64) if live_mask >> l & 1]
    need = [l for l in range(64) if need_mask >> l & 1]
    per = len(live) // g
    writes = []
    if not need:
        return writes, per
    if per == 0:   # each pending lane writes its own group
        for l in need:
            tid = wave * 64 + l
            writes += [(l, c, stage_index(c, tid), None) for c in range(g)]
        return writes, per
    queue = {wave * 64 + k: wave * 64 + l for k, l in enumerate(need)}   # rank -> thread
    for r, l in enumerate(live):
        gj, c = r // g, r % g
        if r >= per * g:
            continue
        qi = wave * 64 + gj
        for b in range(0, len(need), per):
            if b + gj < len(need):
                src_tid = queue[qi + b]
                writes.append((src_tid - wave * 64, c, stage_index(c, src_tid), qi + b))
    return writes, per


@pytest.mark.parametrize("d,elem", [(2, 8), (3, 8), (2, 4), (3, 4), (5, 8), (8, 4), (16, 8),
                                    (16, 4)])
def test_every_chunk_written_once_and_in_bounds(d, elem):
    ch = record_chunks(d, elem)
    g = TAPE_GROUP * ch
    stage_size = TAPE_GROUP * ch * 256
    rng = np.random.default_rng(d * 100 + elem)
    for trial in range(300):
        wave = int(rng.integers(0, 4))
        n_live = int(rng.choice([64, 63, 40, 9, 8, 7, 1, int(rng.integers(1, 65))]))
        live_lanes = sorted(rng.choice(64, n_live, replace=False)) if trial % 3 else list(range(n_live))
        live_mask = sum(1 << int(l) for l in live_lanes)
        p_need = rng.random()
        need_mask = sum(1 << int(l) for l in live_lanes if rng.random() < p_need)
        writes, per = plan(live_mask, need_mask, wave, g)
        need = [l for l in range(64) if need_mask >> l & 1]
        got = {}
        for owner, c, lds, qi in writes:
            assert 0 <= lds < stage_size
            assert lds // 256 == c                       # the owner's chunk c ...
            assert (lds % 256) >> 6 == wave              # ... of this wavefront's lanes
            assert (lds % 256) ^ (c & 7) == wave * 64 + owner
            if qi is not None:
                assert wave * 64 <= qi < wave * 64 + 64   # the wavefront's own queue
            key = (owner, c)
            assert key not in got, "chunk written twice"
            got[key] = True
        assert set(got) == {(l, c) for l in need for c in range(g)}
        if per:
            # one round of stores covers `per` whole groups
            assert per * g <= n_live


def test_conflict_free_reads_of_one_group():
    """The eight chunks of one lane's 32-byte records, read by eight
    neighbouring lanes in one instruction, fall in eight distinct 16-byte
    bank groups (128 bytes of banks), whatever the lane."""
    for tid in range(256):
        groups = {(stage_index(c, tid) * 16 // 16) % 8 for c in range(8)}
        assert len(groups) == 8
    # and the owner's own staging writes, one chunk across 8 neighbouring
    # lanes, also fall in distinct bank groups
    for c in range(8):
        for base in range(0, 256, 8):
            assert len({stage_index(c, base + k) % 8 for k in range(8)}) == 8

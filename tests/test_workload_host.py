"""Host-side layout of a batch (no GPU): the problem table, the buffer offsets the C ABI
reads, and the per-problem gather of the broadening-factor ranks.

A batch crosses strip realizations with the energies of their strip class.  The checks are
invariants of the layout: every problem's blocks are disjoint and in bounds, problems at the
same (class, energy) share one self-energy slot, and the rank of problem p is the rank of
its slot.
"""

import numpy as np
import torch

from paper_1010_2627_amd import inputs, workload


def _batch():
    strips = [inputs.square_strip(W) for W in (3, 5)]
    reals = [workload.Realization(i % 2, inputs.onsite_disorder(strips[i % 2], 2 + i, 1.0, 100 + i))
             for i in range(3)]
    E = [np.array([0.1, 0.2]), np.array([0.3, 0.4, 0.5])]
    return workload.Batch(strips, reals, E, device="cpu"), strips, reals, E


def test_problem_table_layout():
    b, strips, reals, E = _batch()
    h = b.probs.host
    assert b.P == sum(len(E[r.strip]) for r in reals)
    assert b.slice_steps() == sum(int(x) for x in h["L"])
    Ms = np.array([strips[int(s)].M for s in h["strip"]])
    # outputs: disjoint [M][M] blocks in problem order, LDOS: disjoint [L][M] blocks
    ends = h["out_off"] + Ms * Ms
    assert np.all(h["out_off"][1:] == ends[:-1])
    lends = h["ldos_off"] + h["L"] * Ms
    assert np.all(h["ldos_off"][1:] == lends[:-1])
    for p, (ri, ei) in enumerate(b.prob_meta):
        r = reals[int(ri)]
        assert int(h["strip"][p]) == r.strip and int(h["L"][p]) == r.onsite.shape[0]
        assert h["E"][p] == E[r.strip][int(ei)]
        # one self-energy slot per (strip class, energy)
        assert int(h["sigma_off"][p]) == b.sigma_base[r.strip] + int(ei) * Ms[p] * Ms[p]
        assert int(h["sigma_off"][p]) + Ms[p] * Ms[p] <= b.sigma_elems
    # on-site blocks of one realization are shared by its energies and in bounds
    for ri, r in enumerate(reals):
        offs = {int(h["onsite_off"][p]) for p in range(b.P) if int(b.prob_meta[p][0]) == ri}
        assert len(offs) == 1
        assert offs.pop() + r.onsite.size <= b.onsite.numel()


def test_problem_ranks_follow_the_slot():
    b, strips, reals, E = _batch()
    # slot order: class 0's energies, then class 1's
    b.rankL = torch.tensor([7, 8, 20, 21, 22], dtype=torch.int32)
    b.rankR = torch.tensor([1, 2, 3, 4, 5], dtype=torch.int32)
    rl, rr = b.problem_ranks()
    slot_base = [0, len(E[0])]
    for p, (ri, ei) in enumerate(b.prob_meta):
        slot = slot_base[reals[int(ri)].strip] + int(ei)
        assert rl[p] == b.rankL[slot].item() and rr[p] == b.rankR[slot].item()

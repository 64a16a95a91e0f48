"""CPU model of the wait / signal protocol of a shared factorisation (several
work-groups, "ranks", on one subset's Cholesky factor; Sec. 2.3's local
factorisation split across work-groups).

The model lists, for every rank, the steps of the factorisation kernel that
touch memory another rank reads or writes, in the kernel's order:

  per column panel p (columns [c0, c0 + PB)):
    per row chunk of this rank (chunk k of the panel goes to rank k mod R,
    so rank 0 holds the diagonal chunk):
      - before the first update of the panel: wait until the rank-panel
        counter reaches R * p (every rank finished panel p - 1);
      - update: read the panel rows and the chunk rows, columns [0, c0);
      - ranks other than 0, once per panel: wait until the diagonal counter
        reaches p + 1, then read the panel's FP64 diagonal-block inverses;
      - rank 0, diagonal chunk: factor the diagonal blocks, store them and
        their inverses;
      - second 64-column half of a 128-column panel, other chunks: read the
        rows c0 + 64 .. c0 + 128, columns [c0, c0 + 64), from memory;
      - store the chunk's rows of the panel;
      - rank 0, diagonal chunk: set the diagonal counter to p + 1;
    then (R > 1): wait for R * p if not yet done, add one to the rank-panel
    counter;
  ranks other than 0 end; rank 0 waits until the rank-panel counter reaches
  R * panels and writes the log det and status.

Every interleaving of the ranks' steps (exhaustively for up to four ranks,
by random schedules for up to eight) must end with every rank finished
(no deadlock, all ranks resident as the launch arranges) and must never
read a region of L or of the inverses before the rank that writes it has
written it.  Planted mistakes (a dropped wait, a signal before the store, a
counter target one too small) must be caught.
"""
import random

import pytest

WAIT, ADD, SET, READ, WRITE, END = range(6)
TB = 64   # rows per block of the packed factor
RCH = 256  # rows per chunk of the 8-wave work-group


def rank_events(rank, R, npad, PB, drop=None):
    """The protocol steps of one rank, in kernel order.  Regions are
    ("L", row block, panel) and ("inv", 64-column block).  `drop` plants a
    mistake: "inv_wait", "panel_wait", "early_signal" or "short_target"."""
    ev = []
    P = (npad + PB - 1) // PB
    for p in range(P):
        c0 = p * PB
        two = PB == 128 and c0 + 128 <= npad
        synced = R == 1 or c0 == 0
        inv_ready = rank == 0
        for r0 in range(c0 + RCH * rank, npad, RCH * R):
            first = r0 == c0
            rows = range(r0 // TB, min(r0 + RCH, npad) // TB)
            if not synced:
                if drop != "panel_wait":
                    ev.append((WAIT, 1, R * p - (1 if drop == "short_target" else 0)))
                synced = True
            if c0 > 0:
                prow = range(c0 // TB, min(c0 + PB, npad) // TB)
                for b in list(prow) + list(rows):
                    for q in range(p):
                        ev.append((READ, ("L", b, q)))
            if not inv_ready:
                if drop != "inv_wait":
                    ev.append((WAIT, 0, p + 1))
                ev.append((READ, ("inv", c0 // TB)))
                if two:
                    ev.append((READ, ("inv", c0 // TB + 1)))
                inv_ready = True
            if first:
                if drop == "early_signal" and R > 1:
                    ev.append((SET, 0, p + 1))
                ev.append((WRITE, ("inv", c0 // TB)))
                if two:
                    ev.append((WRITE, ("inv", c0 // TB + 1)))
            elif two:
                ev.append((READ, ("L", c0 // TB + 1, p)))
            for b in rows:
                ev.append((WRITE, ("L", b, p)))
            if first and R > 1 and drop != "early_signal":
                ev.append((SET, 0, p + 1))
        if R > 1:
            if not synced and drop != "panel_wait":
                ev.append((WAIT, 1, R * p))
            ev.append((ADD, 1))
    if R > 1 and rank == 0:
        ev.append((WAIT, 1, R * P))
        ev.append((READ, ("status",)))
    ev.append((END,))
    return ev


class Machine:
    def __init__(self, R, npad, PB, drop=None):
        self.ev = [rank_events(r, R, npad, PB, drop) for r in range(R)]
        self.writer = {}
        for r, evs in enumerate(self.ev):
            for i, e in enumerate(evs):
                if e[0] == WRITE:
                    assert e[1] not in self.writer, "a region is written twice"
                    self.writer[e[1]] = (r, i)

    def enabled(self, pcs, ctr):
        out = []
        for r, pc in enumerate(pcs):
            e = self.ev[r][pc]
            if e[0] == END:
                continue
            if e[0] == WAIT and ctr[e[1]] < e[2]:
                continue
            out.append(r)
        return out

    def step(self, pcs, ctr, r):
        """Execute rank r's next step; returns the new state or raises on a
        read before its write."""
        e = self.ev[r][pcs[r]]
        ctr = list(ctr)
        if e[0] == ADD:
            ctr[e[1]] += 1
        elif e[0] == SET:
            ctr[e[1]] = max(ctr[e[1]], e[2])
        elif e[0] == READ and e[1][0] != "status":
            w = self.writer.get(e[1])
            assert w is not None, f"rank {r} reads {e[1]}, which nobody writes"
            if pcs[w[0]] <= w[1]:
                raise RuntimeError(f"rank {r} reads {e[1]} before rank {w[0]} writes it")
        elif e[0] == READ:
            # the status is written after every rank has finished every panel
            if any(self.ev[k][pcs[k]][0] != END for k in range(1, len(pcs))):
                raise RuntimeError("rank 0 finishes before the other ranks")
        pcs = list(pcs)
        pcs[r] += 1
        return tuple(pcs), tuple(ctr)

    def done(self, pcs):
        return all(self.ev[r][pc][0] == END for r, pc in enumerate(pcs))


def explore_all(m):
    """Every interleaving (depth-first over distinct states)."""
    start = (tuple(0 for _ in m.ev), (0, 0))
    seen = {start}
    stack = [start]
    while stack:
        pcs, ctr = stack.pop()
        en = m.enabled(pcs, ctr)
        if not en:
            if not m.done(pcs):
                raise RuntimeError(f"deadlock at {pcs} counters {ctr}")
            continue
        for r in en:
            nxt = m.step(pcs, ctr, r)
            if nxt not in seen:
                seen.add(nxt)
                stack.append(nxt)
    return len(seen)


def run_random(m, seed):
    rnd = random.Random(seed)
    pcs, ctr = tuple(0 for _ in m.ev), (0, 0)
    while True:
        en = m.enabled(pcs, ctr)
        if not en:
            if not m.done(pcs):
                raise RuntimeError(f"deadlock at {pcs} counters {ctr}")
            return
        pcs, ctr = m.step(pcs, ctr, rnd.choice(en))


# padded sizes: whole and ragged panels (multiples of 64), chunks per panel
# from one to several per rank
@pytest.mark.parametrize("PB", [128, 64])
@pytest.mark.parametrize("R,npad", [(1, 640), (2, 576), (2, 1088), (3, 832), (3, 1216), (4, 704)])
def test_every_interleaving_finishes_and_reads_after_writes(R, npad, PB):
    states = explore_all(Machine(R, npad, PB))
    assert states > 0


@pytest.mark.parametrize("R,npad", [(5, 2112), (6, 2560), (8, 3008), (8, 2048), (7, 4032)])
def test_random_schedules_up_to_eight_ranks(R, npad):
    for PB in (128, 64):
        m = Machine(R, npad, PB)
        for seed in range(60):
            run_random(m, seed)


@pytest.mark.parametrize("drop", ["inv_wait", "panel_wait", "early_signal", "short_target"])
def test_planted_protocol_mistakes_are_caught(drop):
    with pytest.raises(RuntimeError):
        explore_all(Machine(2, 704, 128, drop=drop))


def test_the_largest_rank_count_the_launch_uses_matches_the_model():
    """The library gives a shared subset at most 8 work-groups, and sharing
    starts at 2,048 padded rows: at 8 ranks every rank holds a chunk of the
    first panel, at 2,048 rows exactly one each."""
    assert (2048 + RCH - 1) // RCH == 8

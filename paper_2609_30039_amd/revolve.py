"""Binomial checkpoint schedule for the reverse sweep (Section 3.2; Griewank's
binomial checkpointing).

With s checkpoint slots and l steps to reverse, the minimal number of forward
step evaluations is t(l, s) = r l - beta(s+1, r-1), where
beta(s, r) = C(s + r, s) and r is the smallest integer with beta(s, r) >= l.
The recursion below attains it: to reverse steps [a, b) holding u^a in a slot
and as the current state, advance to a + m with
m = max(1, l - beta(s-1, r), beta(s, r-2)) (the upper part then needs at most
r repetitions with s-1 slots and the lower part r-1 repetitions with s slots),
store u^{a+m}, reverse [a+m, b) with one slot fewer, restore u^a and reverse
[a, a+m).  The adjoint of step k reads the current state u^k and
does not re-execute step k.

Actions: ("advance", k) forward k steps; ("save", slot); ("restore", slot);
("adjoint",) one reverse step from m to m-1 (requires the forward state to be
at m-1).
"""
from __future__ import annotations

from math import comb
from typing import List, Tuple

Action = Tuple


def beta(s: int, r: int) -> int:
    if r < 0 or s < 0:
        return 0
    return comb(s + r, s)


def repetitions(l: int, s: int) -> int:
    r = 0
    while beta(s, r) < l:
        r += 1
    return r


def forward_count(l: int, s: int) -> int:
    """Forward steps needed to reverse l steps from u^0 with s slots."""
    if l <= 1:
        return 0
    if s == 1:
        return l * (l - 1) // 2
    r = repetitions(l, s)
    return r * l - beta(s + 1, r - 1)


def schedule(l: int, s: int) -> List[Action]:
    """Actions reversing l steps from u^0 (held in slot 0 and current)."""
    if s < 1:
        raise ValueError("need at least one checkpoint slot")
    out: List[Action] = []
    state = {"t": 0}

    def goto(slot_pos, a):
        if state["t"] != a:
            out.append(("restore", slot_pos))
            state["t"] = a

    def adv(k):
        if k > 0:
            out.append(("advance", k))
            state["t"] += k

    def rev(a: int, b: int, slot_a: int, free: List[int]):
        l_ = b - a
        goto(slot_a, a)
        if l_ == 1:
            out.append(("adjoint",))
            return
        s_ = len(free) + 1
        if s_ == 1:
            for k in range(b - 1, a - 1, -1):
                goto(slot_a, a)
                adv(k - a)
                out.append(("adjoint",))
            return
        r = repetitions(l_, s_)
        m = max(1, l_ - beta(s_ - 1, r), beta(s_, r - 2))
        adv(m)
        slot = free.pop()
        out.append(("save", slot))
        rev(a + m, b, slot, free)
        free.append(slot)
        rev(a, a + m, slot_a, free)

    rev(0, l, 0, list(range(s - 1, 0, -1)))
    return out


def simulate(actions: List[Action], l: int, s: int):
    """Check a schedule: returns (forward steps, adjoint order, max slots used)."""
    t = 0
    m = l
    slots = {0: 0}
    fwd = 0
    order = []
    for a in actions:
        if a[0] == "advance":
            t += a[1]
            fwd += a[1]
        elif a[0] == "save":
            assert 0 <= a[1] < s
            slots[a[1]] = t
        elif a[0] == "restore":
            t = slots[a[1]]
        elif a[0] == "adjoint":
            assert t == m - 1, (t, m)
            order.append(m - 1)
            m -= 1
    assert m == 0
    return fwd, order, len(slots)


def split_recording(actions: List[Action]):
    """Split a schedule into its recording prefix (advances and saves up to the
    first adjoint) and the reverse phase."""
    for q, a in enumerate(actions):
        if a[0] == "adjoint":
            return actions[:q], actions[q:]
    return actions, []

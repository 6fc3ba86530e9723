"""Oracle for the history window rules (Section 4.1, Algorithm 1).

TEST INFRASTRUCTURE ONLY (tests, smoke check and CPU baseline).

After step t: while the window holds fewer than H slices, t is appended;
otherwise j is drawn uniformly from {1..t} and, if j <= H, the j-th element is
replaced by t (reservoir sampling, so the window stays a uniform sample of
the past).  The draw is specified so that two independent implementations
agree: j = (SplitMix64(seed XOR t) mod t) + 1, where SplitMix64(x) is the
first output of Steele, Lea and Flood's SplitMix64 generator started from
state x (add the golden-gamma constant, then the two xor-shift-multiply
rounds and a final xor-shift).
"""
MASK = (1 << 64) - 1


def splitmix64(x: int) -> int:
    z = (x + 0x9E3779B97F4A7C15) & MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def reservoir_draw(seed: int, t: int) -> int:
    """j in {1..t}."""
    return splitmix64((seed ^ t) & MASK) % t + 1


def window_update(slots: list, H: int, t: int, seed: int):
    """slots: list of time stamps in slot order.  Returns (new_slots,
    slot_written or -1) after step t."""
    slots = list(slots)
    if H <= 0:
        return slots, -1
    if len(slots) < H:
        slots.append(t)
        return slots, len(slots) - 1
    j = reservoir_draw(seed, t)
    if j <= H:
        slots[j - 1] = t
        return slots, j - 1
    return slots, -1

"""CPU emulation of the FFA kernel's index arithmetic over the library's real
phase tables and launches (no GPU): every global read and write of every tile
must fall inside its buffer, and every tile may only read what an earlier
launch wrote."""
import ctypes

import numpy as np

from paper_1703_05581_amd import ffa

PHASE_DT = np.dtype([
    ("tile0", "<i8"), ("oct_off", "<i8"), ("first_trial", "<i8"),
    ("ntiles", "<i4"), ("ng", "<i4"), ("step", "<i4"), ("pass_", "<i4"), ("last", "<i4"),
    ("P0", "<i4"), ("M", "<i4"), ("depth", "<i4"), ("D", "<i4"), ("vin", "<i4"),
    ("stride", "<i4"), ("halo", "<i4"), ("wofs", "<i4"), ("nw", "<i4"), ("isqrt_ofs", "<i4"),
    ("launch", "<i4"), ("u16", "<i4"), ("ring64", "<i4")])
assert PHASE_DT.itemsize == 96
SCRATCH = 16 * 64 * 4
LDS_MAX = 160 * 1024
HEADER = 2112

lib = ffa.lib()
lib.ffa_debug_phases.restype = ctypes.c_int64
lib.ffa_debug_phases.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]
lib.ffa_debug_layout.restype = ctypes.c_int64
lib.ffa_debug_layout.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.c_int64]


def phases(plan):
    n = lib.ffa_debug_phases(plan.handle, None, 0)
    arr = np.zeros(n, PHASE_DT)
    assert lib.ffa_debug_phases(plan.handle, arr.ctypes.data, n) == n
    return arr


def layout(plan):
    need = lib.ffa_debug_layout(plan.handle, None, 0)
    out = (ctypes.c_int64 * need)()
    lib.ffa_debug_layout(plan.handle, out, need)
    v = list(out)
    wins = np.array(v[8:], dtype=np.int64).reshape(-1, 4)
    return dict(ring_off=v[0], ring_elems=v[1], n_tiles=v[3], lds_bytes=v[4],
                max_P0=v[5], ws_bytes=v[6], lookahead=v[7], launches=wins)


def octaves(plan):
    """(offset, length) of each octave series: after the header, 64-aligned."""
    out, cur = [], HEADER
    last = max(plan.step(s).f for s in range(plan.n_steps)).bit_length() - 1
    for o in range(last + 1):
        out.append((cur, plan.N >> o))
        cur = (cur + (plan.N >> o) + 63) // 64 * 64
    return out


def check(plan):
    """Walk every launch of a search in order; raise AssertionError on the
    first bad access or ordering."""
    L = layout(plan)
    ph = phases(plan)
    octs = octaves(plan)
    ws_elems = L["ws_bytes"] // 4
    assert L["ring_off"] >= octs[-1][0] + octs[-1][1]
    assert L["ring_off"] + L["ring_elems"] <= ws_elems
    wins = L["launches"]
    assert wins[0, 0] == 0 and int(wins[:, 1].sum()) == L["n_tiles"]
    assert all(wins[i, 0] + wins[i, 1] == wins[i + 1, 0] for i in range(len(wins) - 1))
    done = {}        # (step, pass) -> launch that ran it
    npass = {}       # step -> passes
    for x in ph:
        npass[int(x["step"])] = max(npass.get(int(x["step"]), 0), int(x["pass_"]) + 1)
    live = {}        # step -> (start, end) of the ring range its intermediates hold
    ended = {}       # step -> launch of its last pass
    for x in ph:
        w = int(x["launch"])
        for t in [t for t in live if ended.get(t, w) < w]:
            del live[t]  # read for the last time in an earlier launch
        w0, wn, wlds, wp0 = (int(v) for v in wins[w])
        assert w0 <= x["tile0"] and x["tile0"] + x["ntiles"] <= w0 + wn, "phase outside its launch"
        s, p, P0, M = int(x["step"]), int(x["pass_"]), int(x["P0"]), int(x["M"])
        d, R = int(x["depth"]), 1 << int(x["depth"])
        esz = 2 if x["u16"] else 4
        if x["u16"]:
            # 16-bit rows only on a first pass of a uint8 plan whose sums fit
            octave = plan.step(s).f.bit_length() - 1
            assert p == 0 and not x["last"] and plan.dtype == "u8" and not plan.dered_window, s
            assert 255 * 2 ** (octave + d) < 65536, (s, octave, d)
        lds = R * int(x["stride"]) * esz + (SCRATCH if x["last"] else 0)
        assert lds <= wlds <= LDS_MAX and P0 <= wp0
        MP = M * P0
        region = MP * (2 if npass[s] > 2 else 1)
        slot0 = L["ring_off"] + 64 * int(x["ring64"])
        slot_end = slot0 + region
        if npass[s] > 1:
            assert L["ring_off"] <= slot0 and slot_end <= L["ring_off"] + L["ring_elems"], ("ring range", s)
        if p == 0 and not x["last"]:
            # no step whose intermediates are still to be read holds any of this range
            for t, (a, b) in live.items():
                assert b <= slot0 or slot_end <= a, ("ring range in use", s, t)
            live[s] = (slot0, slot_end)
        if p > 0:
            assert done.get((s, p - 1), w) < w, ("previous pass not in an earlier launch", s, p)
            assert live.get(s) == (slot0, slot_end), ("ring range moved or taken", s)
        Gin = M >> int(x["D"])
        for k in range(int(x["ntiles"])):
            q, h = divmod(k, int(x["ng"]))
            valid = min(R, int(x["vin"]) - (h << d))
            assert valid >= 1
            rel = (q * Gin + (h << d)) * P0
            if p == 0:
                off = int(x["oct_off"])
                n = dict(octs)[off]
                assert 0 <= rel and rel + valid * P0 <= n, ("pass-0 read", s, k)
            else:
                src = slot0 + (MP if (p - 1) & 1 else 0) + rel
                assert slot0 <= src and src + valid * P0 <= slot_end, ("read", s, k)
            if not x["last"]:
                Gout = Gin >> d
                dst = slot0 + (MP if p & 1 else 0) + ((q << d) * Gout + h) * P0
                assert slot0 <= dst and dst + (R - 1) * Gout * P0 + P0 <= slot_end, ("write", s, k)
            else:
                t0 = int(x["first_trial"]) + (q << d)
                assert 0 <= t0 and t0 + R <= plan.n_trials, ("trial", s, k)
        done[(s, p)] = w
        if x["last"]:
            ended[s] = w
    return L

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
    ("launch", "<i4"), ("u16", "<i4"), ("ring64", "<i4"), ("series", "<i4"), ("reserved", "<i4")])
assert PHASE_DT.itemsize == 104
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
    regions = dict(octs)

    def pass0(x):
        return int(x["oct_off"]), regions[int(x["oct_off"])]

    def u16_ok(x, d):
        octave = plan.step(int(x["step"])).f.bit_length() - 1
        return plan.dtype == "u8" and not plan.dered_window and 255 * 2 ** (octave + d) < 65536

    return _check_queue(ph, L, pass0, lambda x: plan.n_trials, u16_ok)


def _check_queue(ph, L, pass0, n_trials, u16_ok):
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
            assert p == 0 and not x["last"] and u16_ok(x, d), s
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
                off, n = pass0(x)
                assert int(x["oct_off"]) == off
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
                assert 0 <= t0 and t0 + R <= n_trials(x), ("trial", s, k)
        done[(s, p)] = w
        if x["last"]:
            ended[s] = w
    return L


lib.ffa_debug_batch.restype = ctypes.c_int64
lib.ffa_debug_batch.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64,
                                ctypes.POINTER(ctypes.c_int64), ctypes.c_int64]
lib.ffa_debug_batch_series_base.restype = ctypes.c_int64
lib.ffa_debug_batch_series_base.argtypes = [ctypes.c_void_p, ctypes.c_int32]


def batch_queue(batch, c):
    """Phases and layout of class c of a batch (None past the last class)."""
    n = lib.ffa_debug_batch(batch.handle, c, None, 0, None, 0)
    if n < 0:
        return None
    arr = np.zeros(n, PHASE_DT)
    lib.ffa_debug_batch(batch.handle, c, arr.ctypes.data, n, None, 0)
    need = 8 + 4 * 100000
    out = (ctypes.c_int64 * need)()
    lib.ffa_debug_batch(batch.handle, c, None, 0, out, need)
    nl = int(np.unique(arr["launch"]).max()) + 1 if n else 0
    v = list(out[: 8 + 4 * nl])
    wins = np.array(v[8:], dtype=np.int64).reshape(-1, 4)
    L = dict(ring_off=v[0], ring_elems=v[1], n_classes=v[2], n_tiles=v[3], lds_bytes=v[4], max_P0=v[5],
             ws_bytes=v[6], lookahead=v[7], launches=wins)
    return arr, L


def check_batch(batch):
    """check() for every class queue of a batch: each series reads only its
    own octave series (in its region of the batch workspace) and writes only
    its own trials; the classes' rings lie apart and inside the workspace."""
    bases = [lib.ffa_debug_batch_series_base(batch.handle, i) for i in range(len(batch.plans))]
    ends = bases[1:] + [None]
    per = []
    for i, p in enumerate(batch.plans):
        octs = {bases[i] + off: n for off, n in octaves(p)}
        per.append(octs)
    rings = []
    out = []
    c = 0
    while True:
        got = batch_queue(batch, c)
        if got is None:
            break
        ph, L = got
        assert L["ring_off"] >= bases[-1] and L["ring_off"] + L["ring_elems"] <= L["ws_bytes"] // 4
        rings.append((L["ring_off"], L["ring_off"] + L["ring_elems"]))

        def pass0(x):
            i = int(x["series"])
            off = int(x["oct_off"])
            assert off in per[i], ("octave series of another series", i, off)
            if ends[i] is not None:
                assert off + per[i][off] <= ends[i]
            return off, per[i][off]

        def u16_ok(x, d):
            p = batch.plans[int(x["series"])]
            f = [p.step(s).f for s in range(p.n_steps) if p.step(s).first_trial == int(x["first_trial"])][0]
            return p.dtype == "u8" and not p.dered_window and 255 * 2 ** (f.bit_length() - 1 + d) < 65536

        out.append(_check_queue(ph, L, pass0, lambda x: batch.plans[int(x["series"])].n_trials, u16_ok))
        c += 1
    rings.sort()
    assert all(a[1] <= b[0] for a, b in zip(rings, rings[1:])), rings
    return out

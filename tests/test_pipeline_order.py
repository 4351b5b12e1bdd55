"""The ordering of the bench's pipelined schedule, on the CPU with recording
stand-ins for streams, events and the library calls: every write to a
workspace waits for the last reader of what it overwrites, and every
backtrace starts after its own DP."""
import pytest

import bench


class Event:
    def __init__(self, log, name):
        self.log, self.name, self.stream = log, name, None

    def record(self, stream):
        self.stream = stream
        self.log.append(("record", stream.name, self.name))


class Stream:
    def __init__(self, log, name):
        self.log, self.name = log, name

    def wait_event(self, ev):
        self.log.append(("wait", self.name, ev.name))


class Lib:
    """The pardtw calls bench.launch_pipelined makes, logged with their stream and workspace."""
    PREC_F32 = 0
    LAYOUT_PANEL_BAND = 2

    def __init__(self, log):
        self.log = log
        self.count = {}

    def _call(self, kind, w, stream):
        # calls of one kind are issued in step order: the i-th belongs to pair i
        i = self.count.get(kind, 0)
        self.count[kind] = i + 1
        self.log.append(("call", stream.name, kind, w.name, i))

    def pardtw_cost(self, X, Y, C, prec, layout, stream):
        self._call("cost", C.owner, stream)

    def pardtw_dp(self, C, n, m, bp, total, status, ws, layout, stream):
        self._call("dp", bp.owner, stream)

    def pardtw_dp_fused(self, X, Y, bp, total, status, ws, stream):
        self._call("dp", bp.owner, stream)

    def pardtw_dp_packed(self, C, n, m, bp, total, status, ws, layout, stream):
        self._call("dp_packed", bp.owner, stream)

    def pardtw_dp_fused_packed(self, X, Y, bp, total, status, ws, stream):
        self._call("dp_packed", bp.owner, stream)

    def pardtw_backtrace_packed(self, bp, n, m, status, path, path_len, stream):
        self._call("bt_packed", bp.owner, stream)

    def pardtw_backtrace_parallel(self, bp, n, m, status, path, path_len, ws, stream, packed):
        assert ws.owner is bp.owner
        self._call("bt_packed" if packed else "bt", bp.owner, stream)

    def pardtw_dp_fused_ckpt(self, X, Y, K, ckpt, total, status, ws, stream):
        self._call("dp", ckpt.owner, stream)

    def pardtw_backtrace(self, bp, n, m, status, path, path_len, stream):
        self._call("bt", bp.owner, stream)

    def pardtw_ckpt_backtrace(self, X, Y, K, ckpt, status, path, path_len, stream):
        self._call("bt", ckpt.owner, stream)

    def pardtw_ckpt_backtrace_parallel(self, X, Y, K, ckpt, status, path, path_len, ws, stream):
        assert ws.owner is ckpt.owner
        self._call("bt", ckpt.owner, stream)


class Buf:
    def __init__(self, owner):
        self.owner = owner


class Workspace:
    def __init__(self, name, packed=False):
        self.name = name
        self.packed = packed
        for f in ("C", "bp", "ckpt", "total", "status", "ws", "path", "path_len", "bt_ws"):
            setattr(self, f, Buf(self))


class Shape:
    shape = (100, 12)


@pytest.mark.parametrize("fused,K,packed", [(False, 0, False), (True, 0, False), (False, 64, False),
                                            (False, 0, True), (True, 0, True)])
@pytest.mark.parametrize("nbuf,nbt", [(2, 1), (3, 2), (2, 2)])
@pytest.mark.parametrize("serial_walk", [False, True])
def test_pipelined_order(fused, K, packed, nbuf, nbt, serial_walk):
    log = []
    steps = 9
    stream = Stream(log, "main")
    bts = [Stream(log, f"bt{i}") for i in range(nbt)]
    bufs = [Workspace(f"w{i}", packed) for i in range(nbuf)]
    dp_kind, bt_kind = ("dp_packed", "bt_packed") if packed else ("dp", "bt")
    evs = [[Event(log, (s, k)) for k in range(6)] for s in range(steps)]
    bench.launch_pipelined(Lib(log), Shape(), Shape(), bufs, stream, (stream, bts), steps, fused, K, evs,
                           serial_walk=serial_walk)

    def pos(entry):
        return log.index(entry)

    for s in range(steps):
        w = f"w{s % nbuf}"
        s_bt = f"bt{s % nbt}"
        dp = pos(("call", "main", dp_kind, w, s))
        bt = pos(("call", s_bt, bt_kind, w, s))
        # the backtrace waits on this pair's DP end event, recorded after the DP call
        dp_end = pos(("record", "main", (s, 3)))
        assert dp < dp_end < pos(("wait", s_bt, (s, 3))) < bt
        if not fused and not K:
            cost = pos(("call", "main", "cost", w, s))
            assert pos(("wait", "main", (s, 1))) < dp and cost < dp
        if s >= nbuf:
            # the DP rewrites this workspace's codes (or checkpoints) only after
            # the backtrace of pair s - nbuf, which read them, has ended
            prev_bt_end = pos(("record", f"bt{(s - nbuf) % nbt}", (s - nbuf, 5)))
            assert prev_bt_end < pos(("wait", "main", (s - nbuf, 5))) < dp
            assert pos(("call", f"bt{(s - nbuf) % nbt}", bt_kind, w, s - nbuf)) < prev_bt_end
            if not fused and not K:
                # and the cost matrix only after the DP of pair s - nbuf, which read it
                assert pos(("wait", "main", (s - nbuf, 3))) < pos(("call", "main", "cost", w, s))

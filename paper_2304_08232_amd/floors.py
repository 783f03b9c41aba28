"""Device floors behind the design of the coarse levels (measurement only).

measure(torch) returns, on the current device:
  empty_launch_us     per launch of an empty kernel, back to back on one
                      stream: issued eagerly, and replayed from a captured
                      graph, for a 1-workgroup and a 512-workgroup grid;
  one_shot_read_us    one launch of the streaming-read kernel over 10 MB,
                      79 MB, 489 MB and 4 GB (a level-1 pass, a level-0
                      pass and the CG product at 128^3 move about the first
                      three): the time a kernel that only streams that many
                      bytes takes, ramp-up and drain included;
  barrier_round_us    per round of a barrier among the workgroups of one
                      persistent launch: all 256 workgroups (one per CU,
                      every XCD), or 32 workgroups of one XCD; with agent-scope
                      release/acquire fences around the flag exchange
                      ("fenced": ordinary loads and stores carry the data), or
                      the flag exchange alone ("relaxed": the data would have
                      to travel as agent-scope atomics).
The kernels are in csrc/ceiling.hip (libceiling.so).
"""
import ctypes as C


def _lib():
    from paper_2304_08232_amd import build as libbuild
    L = C.CDLL(libbuild.CEILING_LIB)
    L.ceiling_empty.restype = C.c_int
    L.ceiling_empty.argtypes = [C.c_int, C.c_int, C.c_void_p]
    L.ceiling_barrier.restype = C.c_int
    L.ceiling_barrier.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_longlong,
                                  C.c_void_p]
    return L


def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def empty_launch_us(torch, blocks, launches=2000, graph=False):
    L = _lib()
    stream = torch.cuda.current_stream()

    def issue(st):
        for _ in range(launches):
            rc = L.ceiling_empty(blocks, 64, C.c_void_p(st.cuda_stream))
            if rc != 0:
                raise RuntimeError(f"ceiling_empty failed: {rc}")

    if graph:
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        with torch.cuda.stream(side):
            with torch.cuda.graph(g, stream=side):
                issue(side)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        e0, e1 = _events(torch)
        e0.record(stream)
        g.replay()
        e1.record(stream)
        e1.synchronize()
    else:
        issue(stream)
        torch.cuda.synchronize()
        # queue the launches behind a spin so the host's issue rate is hidden
        torch.cuda._sleep(20_000_000)
        e0, e1 = _events(torch)
        e0.record(stream)
        issue(stream)
        e1.record(stream)
        e1.synchronize()
    return e0.elapsed_time(e1) * 1e3 / launches


def barrier_round_us(torch, kind, blocks, stride, rounds=2000, spin_limit=1 << 22):
    L = _lib()
    stream = torch.cuda.current_stream()
    parts = (blocks + stride - 1) // stride
    flags = torch.zeros(parts, dtype=torch.int32, device="cuda")
    err = torch.zeros(1, dtype=torch.int32, device="cuda")

    def run(nr):
        flags.zero_()
        rc = L.ceiling_barrier(kind, blocks, stride, nr, C.c_void_p(flags.data_ptr()), C.c_void_p(err.data_ptr()),
                               spin_limit, C.c_void_p(stream.cuda_stream))
        if rc != 0:
            raise RuntimeError(f"ceiling_barrier failed: {rc}")

    run(10)
    torch.cuda.synchronize()
    e0, e1 = _events(torch)
    t = {}
    for nr in (rounds // 10, rounds):
        flags.zero_()
        e0.record(stream)
        run(nr)
        e1.record(stream)
        e1.synchronize()
        t[nr] = e0.elapsed_time(e1) * 1e3
    if int(err.item()) != 0:
        raise RuntimeError("barrier probe: a wait exceeded its spin limit")
    # the difference of two round counts removes the launch itself
    return (t[rounds] - t[rounds // 10]) / (rounds - rounds // 10)


def one_shot_read_us(torch, nbytes, reps=20):
    """Time of one launch of the streaming-read kernel over `nbytes` (the
    best grid of 1024..8192 workgroups, the best of `reps` back-to-back
    launches each timed by its own events): what a kernel that only reads
    that many bytes once takes from launch to end, ramp-up and drain
    included."""
    import ctypes as C
    from paper_2304_08232_amd import build as libbuild
    L = C.CDLL(libbuild.CEILING_LIB)
    L.ceiling_stream_read.restype = C.c_int
    L.ceiling_stream_read.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_int, C.c_void_p]
    n16 = nbytes // 16
    buf = torch.zeros(2 * n16, dtype=torch.float64, device="cuda")
    out = torch.zeros(1 << 14, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    best = 1e30
    for blocks in (1024, 2048, 4096, 8192):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * reps)]
        torch.cuda._sleep(20_000_000)
        for k in range(reps):
            ev[2 * k].record(stream)
            rc = L.ceiling_stream_read(C.c_void_p(buf.data_ptr()), n16, C.c_void_p(out.data_ptr()), blocks,
                                       C.c_void_p(stream.cuda_stream))
            ev[2 * k + 1].record(stream)
            if rc != 0:
                raise RuntimeError(f"ceiling_stream_read failed: {rc}")
        torch.cuda.synchronize()
        for k in range(reps):
            best = min(best, ev[2 * k].elapsed_time(ev[2 * k + 1]) * 1e3)
    del buf, out
    return best


def measure(torch):
    out = {"empty_launch_us": {}, "barrier_round_us": {}, "one_shot_read_us": {}}
    for mb in (10, 79, 489, 4096):
        t = one_shot_read_us(torch, mb * 10 ** 6)
        out["one_shot_read_us"][f"{mb}MB"] = {"us": round(t, 3), "gbs": round(mb * 1e6 / t / 1e3, 1)}
    for blocks in (1, 512):
        for graph in (False, True):
            key = f"{blocks}wg_{'graph' if graph else 'eager'}"
            out["empty_launch_us"][key] = round(empty_launch_us(torch, blocks, graph=graph), 3)
    for kind, name in ((0, "fenced"), (1, "relaxed")):
        out["barrier_round_us"][f"{name}_256wg_all_xcds"] = round(barrier_round_us(torch, kind, 256, 1), 3)
        out["barrier_round_us"][f"{name}_32wg_one_xcd"] = round(barrier_round_us(torch, kind, 256, 8), 3)

    return out


if __name__ == "__main__":
    import json
    import torch
    print(json.dumps(measure(torch)))

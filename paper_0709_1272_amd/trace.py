"""Export of the scheduler's task trace (tileqr_trace) as a Chrome trace-event
JSON file, which Perfetto (ui.perfetto.dev) and chrome://tracing open: one
row per workgroup, one slice per task (its body), with the fence and
successor-update time and the queue wait as separate slices.  This is the
execution-flow view of the paper's DAG scheduling (Section 4): which worker
ran which task when.

    from paper_0709_1272_amd import tileqr, trace
    ... tileqr.factor(..., tileqr.opts(flags=tileqr.FLAG_TRACE)) ...
    events, hz = tileqr.trace()
    trace.write_chrome_json("qr.json", events, hz)

Host-side formatting only: the events come from the library's device trace.
"""
import json

KIND = {0: "GEQRT", 1: "TSQRT", 2: "LARFB", 3: "SSRFB", 4: "PUPD"}


def task_name(ev):
    """'SSRFB(k,i,j) s' style label of one event tuple (type, k, i, j, strip,
    worker, t_pop, t_start, t_body_end, t_end)."""
    typ, k, i, j, strip = ev[:5]
    kind = KIND.get(typ, f"T{typ}")
    if typ in (0, 1):                    # the strip field holds the inner panel
        return f"{kind}({k},{i}) panel {strip}"
    if typ == 4:                         # j holds the inner panel
        return f"{kind}({k},{i}) panel {j} strip {strip}"
    return f"{kind}({k},{i},{j}) strip {strip}"


def chrome_events(events, clock_hz):
    """Trace-event dicts (complete events, microseconds from the first pop)."""
    if not events:
        return []
    t0 = min(ev[6] for ev in events)
    us = 1e6 / float(clock_hz)
    out = []
    workers = sorted({ev[5] for ev in events})
    for w in workers:
        role, wg = w >> 16, w & 0xFFFF
        out.append({"ph": "M", "name": "thread_name", "pid": 0, "tid": w,
                    "args": {"name": f"{'panel' if role == 0 else 'update'} wg {wg}"}})
        out.append({"ph": "M", "name": "thread_sort_index", "pid": 0, "tid": w, "args": {"sort_index": w}})
    for ev in events:
        typ, k, i, j, strip, w, t_pop, t_start, t_body, t_end = ev[:10]
        name = task_name(ev)
        args = {"k": k, "i": i, "j": j, "strip": strip}
        if t_start > t_pop:
            out.append({"ph": "X", "name": "acquire", "cat": "fence", "pid": 0, "tid": w,
                        "ts": (t_pop - t0) * us, "dur": (t_start - t_pop) * us, "args": {"task": name}})
        out.append({"ph": "X", "name": name, "cat": KIND.get(typ, "task"), "pid": 0, "tid": w,
                    "ts": (t_start - t0) * us, "dur": max(t_body - t_start, 0) * us, "args": args})
        if t_end > t_body:
            out.append({"ph": "X", "name": "release + successors", "cat": "fence", "pid": 0, "tid": w,
                        "ts": (t_body - t0) * us, "dur": (t_end - t_body) * us, "args": {"task": name}})
    return out


def write_chrome_json(path, events, clock_hz):
    """Write the trace to `path`; returns the number of trace events."""
    ev = chrome_events(events, clock_hz)
    with open(path, "w") as f:
        json.dump({"traceEvents": ev, "displayTimeUnit": "ms"}, f)
    return len(ev)

"""Scan of gfx950 device assembly for workgroup barriers that a wave can reach
while one of its own LDS operations is still outstanding.

On gfx950 s_barrier does not wait for the issuing wave's LDS traffic, so every
barrier that orders LDS accesses between waves must be preceded, on every path
into it, by s_waitcnt lgkmcnt(0).  The scan splits each kernel into basic
blocks, propagates "an LDS access may be outstanding" along the control-flow
edges (branches, fall-through, loop back-edges) to a fixed point, and reports
each s_barrier reached with that flag set.  Cross-lane DS instructions
(ds_bpermute, ds_permute, ds_swizzle) touch no LDS memory and are ignored; only
lgkmcnt(0) clears the flag, so the scan is conservative."""
import re
from collections import defaultdict

_CROSS_LANE = re.compile(r"ds_(bpermute|permute|swizzle)")


def kernels(text):
    """(symbol, body lines) of every function in an assembly file."""
    cur, lines = None, []
    for ln in text.splitlines():
        m = re.match(r"^(_Z\S+):", ln)
        if m:
            if cur:
                yield cur, lines
            cur, lines = m.group(1), []
            continue
        if cur and ln.startswith(".Lfunc_end"):
            yield cur, lines
            cur, lines = None, []
            continue
        if cur is not None:
            lines.append(ln)


def _blocks(lines):
    blocks, order = {}, []
    cur = "__entry"
    blocks[cur] = []
    order.append(cur)
    for ln in lines:
        code = ln.split(";")[0].strip()
        if not code:
            m = re.match(r"^;\s*(%bb\.\d+):", ln.strip())
            if m:
                cur = m.group(1)
                blocks[cur] = []
                order.append(cur)
            continue
        m = re.match(r"^(\.LBB\S+):", code)
        if m:
            cur = m.group(1)
            blocks[cur] = []
            order.append(cur)
            continue
        if code.startswith("."):
            continue
        blocks[cur].append(code)
        if code.split()[0] == "s_branch" or code.split()[0].startswith("s_cbranch"):
            cur = f"__after{len(order)}"  # code after a branch starts a block
            blocks[cur] = []
            order.append(cur)
    succ = defaultdict(list)
    for i, b in enumerate(order):
        ins = blocks[b]
        nxt = order[i + 1] if i + 1 < len(order) else None
        last = ins[-1].split() if ins else [""]
        if last[0] == "s_branch":
            succ[b].append(last[1])
        elif last[0].startswith("s_cbranch"):
            succ[b].append(last[1])
            if nxt:
                succ[b].append(nxt)
        elif last[0] in ("s_endpgm", "s_setpc_b64"):
            pass
        elif nxt:
            succ[b].append(nxt)
    return blocks, order, succ


def _step(ins, pending):
    op = ins.split()[0]
    if op.startswith("ds_") and not _CROSS_LANE.match(op):
        return True
    if op == "s_waitcnt" and "lgkmcnt(0)" in ins:
        return False
    return pending


def unsafe_barriers(lines):
    """[(block, index)] of barriers reachable with an LDS access outstanding, and
    the number of barriers in the function."""
    blocks, order, succ = _blocks(lines)
    pend = {b: False for b in order}
    changed = True
    while changed:
        changed = False
        for b in order:
            p = pend[b]
            for ins in blocks[b]:
                p = _step(ins, p)
            if p:
                for t in succ[b]:
                    if t in pend and not pend[t]:
                        pend[t] = True
                        changed = True
    found, nbar = [], 0
    for b in order:
        p = pend[b]
        for k, ins in enumerate(blocks[b]):
            if ins.split()[0] == "s_barrier":
                nbar += 1
                if p:
                    found.append((b, k))
            p = _step(ins, p)
    return found, nbar

"""Audit of workgroup barriers in gfx950 assembly: a barrier must never sit where the execution
mask may have been narrowed by divergent control flow.

On AMD GPUs a branch whose condition is not provably wave-uniform is compiled as an exec-masked
region (s_and_saveexec / s_or_b64 exec, exec, ...), and a loop with such an exit keeps narrowing
exec (s_andn2_b64 exec, exec, ...).  A wave whose mask becomes empty skips the region, so a barrier
inside it is reached a different number of times by different waves and the workgroup hangs.

The audit walks each function's control-flow graph and tracks, per basic block, the set of
mask registers whose divergent region is open (entered by a save-exec or an exec-narrowing loop
latch, closed by the matching `s_or_b64 exec, exec, sX`, which also closes the regions nested in it, or an exec
restore).  The state at a merge keeps every region open on any predecessor (conservative).  A barrier, or a call, reached with a
non-empty set is reported.
"""
from __future__ import annotations

import re
import subprocess

_LABEL = re.compile(r"^(\.LBB\d+_\d+):")
_BB = re.compile(r"^; %bb\.\d+:")
_FUNC = re.compile(r"^([A-Za-z_][\w.$]*):\s*(;.*)?$")
_SREG = r"(s\[\d+:\d+\]|vcc|s\d+)"


def compile_to_asm(src: str, out: str, extra=()):
    cmd = ["hipcc", "-O3", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "--cuda-device-only", "-S", src, "-o", out] + list(extra)
    subprocess.check_call(cmd, stderr=subprocess.DEVNULL)
    return open(out).read()


def functions(asm: str):
    """Yields (name, [instruction lines]) for every function body in the assembly."""
    name, body = None, []
    for raw in asm.splitlines():
        line = raw.split("//")[0].rstrip()
        m = _FUNC.match(line)
        if m and not line.startswith(".") and "@" not in m.group(1):
            if name:
                yield name, body
            name, body = m.group(1), []
            continue
        if name is None:
            continue
        if line.startswith(".Lfunc_end"):
            yield name, body
            name, body = None, []
            continue
        s = line.strip()
        if not s or (s.startswith(";") and not _BB.match(s)) or (s.startswith(".") and not _LABEL.match(s)):
            continue
        body.append(s)
    if name:
        yield name, body


def blocks(body):
    """Splits a body into basic blocks: [(label or None, [insns], [successor labels], falls_through)]."""
    out, cur, label = [], [], None
    auto = 0

    def close(fall):
        nonlocal cur, label
        out.append([label, cur, [], fall])
        cur, label = [], None

    for s in body:
        m = _LABEL.match(s)
        if m or _BB.match(s):
            if cur or label is not None:
                close(True)
            if m:
                label = m.group(1)
            else:
                auto += 1
                label = f"%auto{auto}"
            continue
        cur.append(s)
        op = s.split()[0]
        if op == "s_branch":
            out_lbl = s.split()[1]
            close(False)
            out[-1][2].append(out_lbl)
        elif op.startswith("s_cbranch"):
            out_lbl = s.split()[1]
            close(True)
            out[-1][2].append(out_lbl)
        elif op in ("s_endpgm", "s_setpc_b64", "s_trap"):
            close(False)
    if cur or label is not None:
        close(False)
    return out


# The state is a stack of entries (kind, register): ("narrow", r) marks a region in which exec may
# be a strict subset of the mask on entry, to be closed by `s_or_b64 exec, exec, r`; ("mark", r)
# records that r holds a saved copy of exec (`s_mov_b64 r, exec`), which a later
# `s_or_b64 exec, exec, r` or `s_mov_b64 exec, r` restores.  Regions are nested: closing one closes
# everything opened inside it.
def _find(st, reg):
    for i in range(len(st) - 1, -1, -1):
        if st[i][1] == reg:
            return i
    return -1


def _push(st, kind, reg):
    i = _find(st, reg)
    if i >= 0:                      # re-entering a region (a loop latch): drop what it enclosed
        return st[:i] + ((kind, reg),)
    return st + ((kind, reg),)


def _close(st, reg):
    i = _find(st, reg)
    if i < 0:
        return st
    return st[:i]


def _restore(st, reg):
    i = _find(st, reg)
    if i < 0:
        return None
    return st[:i + 1] if st[i][0] == "mark" else st[:i]


def _halves(reg):
    """'s[4:5]' -> ('s4', 's5'); None for anything else."""
    m = re.match(r"^s\[(\d+):(\d+)\]$", reg)
    if not m or int(m.group(2)) != int(m.group(1)) + 1:
        return None
    return f"s{m.group(1)}", f"s{m.group(2)}"


def spill_slots(body):
    """Lane slots of SGPR spills: (vgpr, lane) -> the set of SGPRs ever written there."""
    slots = {}
    for s in body:
        parts = s.replace(",", " ").split()
        if parts[0] == "v_writelane_b32" and len(parts) >= 4:
            slots.setdefault((parts[1], parts[3]), set()).add(parts[2])
    return slots


_NOWRITE = ("s_cbranch", "s_branch", "s_waitcnt", "s_barrier", "s_nop", "s_sleep", "s_setprio", "s_endpgm",
            "s_store", "s_buffer_store", "s_dcache", "s_trap", "s_setpc", "s_swappc", "s_call", "s_cmp",
            "s_bitcmp", "s_set_gpr_idx")


def _sregs(reg):
    """The 32-bit SGPR names a register operand covers ('s[4:5]' -> {'s4', 's5'})."""
    m = re.match(r"^s\[(\d+):(\d+)\]$", reg)
    if m:
        return {f"s{i}" for i in range(int(m.group(1)), int(m.group(2)) + 1)}
    return {reg} if re.match(r"^s\d+$", reg) else set()


def _written_sregs(op, parts):
    """SGPRs an instruction writes through its first operand (scalar ALU results, 64-bit compare
    masks, lane reads); empty for stores, branches and the like."""
    if len(parts) < 2:
        return set()
    if op.startswith("s_") and not op.startswith(_NOWRITE):
        return _sregs(parts[1])
    if op.startswith(("v_cmp", "v_readfirstlane", "v_readlane")) and (op.endswith("_e64") or "readlane" in op
                                                                       or "readfirstlane" in op):
        return _sregs(parts[1])
    return set()


def transfer(insns, state, findings, where, slots=None):
    st = tuple(state)
    anded = {}      # this block: s_and_b64 dst, <saved exec>, x  ->  dst: the saved exec register
    reread = {}     # this block: v_readlane_b32 sM, v, lane from a slot with one spilled SGPR
    for s in insns:
        parts = s.replace(",", " ").split()
        op = parts[0]
        # a saved copy of exec is gone once its register is overwritten (the instruction's own
        # effect on the state is applied below)
        w = _written_sregs(op, parts)
        if w:
            st = tuple(e for e in st if not (e[0] == "mark" and _sregs(e[1]) & w))
        if op == "v_readlane_b32" and len(parts) >= 4 and slots is not None:
            src = slots.get((parts[2], parts[3]), set())
            if len(src) == 1:
                reread[parts[1]] = next(iter(src))
            else:
                reread.pop(parts[1], None)
            continue
        if op == "s_and_b64" and len(parts) >= 4 and parts[1] != "exec":
            for cand in (parts[2], parts[3]):
                i = _find(st, cand)
                if i >= 0 and st[i][0] == "mark":
                    anded[parts[1]] = cand
                    break
            else:
                anded.pop(parts[1], None)
        if op == "s_or_b64" and len(parts) >= 4 and parts[1] == "exec" and parts[2] == "exec" \
                and _find(st, parts[3]) < 0:
            # exec restored from a copy that went through a spill slot: the saved register it was
            # spilled from closes the region
            h = _halves(parts[3])
            if h and h[0] in reread and h[1] in reread:
                lo, hi = reread[h[0]], reread[h[1]]
                if lo.startswith("s") and hi.startswith("s") and lo[1:].isdigit() and hi[1:].isdigit() \
                        and int(hi[1:]) == int(lo[1:]) + 1:
                    parts = parts[:3] + [f"s[{lo[1:]}:{hi[1:]}]"]
        if op == "s_mov_b64" and len(parts) >= 3 and parts[1] == "exec" and parts[2] in anded:
            # exec = saved & cond: a region closed by restoring the saved register
            st = _push(st, "narrow", anded[parts[2]])
            continue
        if op == "s_barrier" or op.startswith("s_swappc") or op == "s_call_b64":
            narrowed = [r for k, r in st if k == "narrow"]
            if narrowed:
                findings.append((where, s, narrowed))
        elif op == "s_or_saveexec_b64" and len(parts) > 2 and parts[2] == "-1":
            st = _push(st, "mark", parts[1])     # whole-wave section (a register spill): exec saved
        elif op in ("s_andn2_saveexec_b64", "s_or_saveexec_b64") and len(parts) > 2 \
                and _find(st, parts[2]) >= 0 and st[_find(st, parts[2])][0] == "narrow":
            # the other arm of an if/else: the source holds that arm's lanes (see the s_xor_b64
            # rule below), the destination saves the lanes of the arm just run, and
            # `s_or_b64 exec, exec, dst` after the other arm closes the whole if/else
            i = _find(st, parts[2])
            st = st[:i] + (("narrow", parts[1]),) + st[i + 1:]
        elif op in ("s_and_saveexec_b64", "s_andn2_saveexec_b64", "s_or_saveexec_b64", "s_xor_saveexec_b64"):
            st = _push(st, "narrow", parts[1])
        elif op == "s_or_b64" and len(parts) >= 4 and parts[1] == "exec" and parts[2] == "exec":
            st = _close(st, parts[3])
        elif op == "s_xor_b64" and len(parts) >= 4 and parts[1] != "exec" and parts[2] == "exec":
            # x = exec ^ saved: the lanes of the other arm; `s_or_b64 exec, exec, x` then closes the
            # region that `saved` opened
            i = _find(st, parts[3])
            if i >= 0:
                st = st[:i] + ((st[i][0], parts[1]),) + st[i + 1:]
        elif op in ("s_andn2_b64", "s_and_b64") and len(parts) >= 4 and parts[1] == "exec":
            st = _push(st, "narrow", parts[3] if parts[3] != "exec" else parts[2])
        elif op == "s_mov_b64" and len(parts) >= 3:
            if parts[1] == "exec":
                if parts[2] in ("-1", "0xffffffffffffffff"):
                    pass                         # whole-wave section, undone by the restore after it
                else:
                    r = _restore(st, parts[2])
                    st = r if r is not None else _push(st, "narrow", "exec<-" + parts[2])
            elif parts[2] == "exec":
                st = _push(st, "mark", parts[1])
    return st


def _merge(a, b):
    if a is None:
        return b
    if a[:len(b)] == b:
        return a
    if b[:len(a)] == a:
        return b
    return a + tuple(x for x in b if x not in a)


def audit(asm: str):
    """Returns [(function, block, instruction, open registers)] for every barrier or call that
    may run under a narrowed execution mask."""
    findings = []
    for fname, body in functions(asm):
        bl = blocks(body)
        if not bl:
            continue
        slots = spill_slots(body)
        index = {b[0]: i for i, b in enumerate(bl) if b[0]}
        succ = []
        for i, (lbl, insns, targets, fall) in enumerate(bl):
            s = [index[t] for t in targets if t in index]
            if fall and i + 1 < len(bl):
                s.append(i + 1)
            succ.append(s)
        state_in = [None] * len(bl)
        state_in[0] = ()
        work = [0]
        while work:
            i = work.pop()
            out = transfer(bl[i][1], state_in[i], [], None, slots)
            for j in succ[i]:
                new = _merge(state_in[j], out)
                if new != state_in[j]:
                    state_in[j] = new
                    work.append(j)
        for i, b in enumerate(bl):
            if state_in[i] is not None:
                transfer(b[1], state_in[i], findings, (fname, b[0]), slots)
    return [(w[0], w[1], s, regs) for (w, s, regs) in findings]

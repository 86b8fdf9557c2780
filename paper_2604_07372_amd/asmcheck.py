"""Build-time check of the generated gfx950 assembly.

A divergent `if` compiles to: narrow exec (s_and_saveexec_b64), skip the body
when no lane is left (s_cbranch_execz JOIN), body, then at JOIN restore exec
(s_or_b64 exec, exec, ...).  Register copies or spill stores placed between the
JOIN label and that restore run with the narrowed mask, so lanes outside the
`if` silently skip them.  Such code was seen for kernels whose masked tail used
exec-masked loads under high register pressure, and it corrupted the ragged
lane's data; the kernels are written to avoid divergent branches around live
state, and this check makes sure no generated kernel has the pattern again.

Only vector work counts: lane reads/writes (v_readlane, v_writelane,
v_readfirstlane) ignore exec, and scalar instructions are not masked.  A join
block of an if / else first switches exec to the else lanes
(s_andn2_saveexec_b64); vector work after that switch is the else branch's
own, not the pattern.
"""
from __future__ import annotations

import re
import sys

__all__ = ["find_masked_joins", "check_files"]

_LABEL = re.compile(r"^(\.LBB\w+):")
_FUNC = re.compile(r"^(_Z\w+):")
_NARROW = re.compile(r"^s_(and|andn2|or|xor|orn2|nand|nor|xnor)_saveexec_b64\b|^s_\w+_b64 exec,|^s_mov_b64 exec,")
_EXECZ = re.compile(r"^s_cbranch_execz (\.LBB\w+)")
_LANE_OPS = ("v_writelane", "v_readlane", "v_readfirstlane")
_VECTOR = ("v_", "scratch_", "global_", "buffer_", "ds_", "flat_")


def _is_restore(t: str) -> bool:
    return t.startswith("s_or_b64 exec, exec") or t.startswith("s_mov_b64 exec, -1")


def find_masked_joins(text: str) -> list[tuple[str, int, list[str]]]:
    """(function, line, first offending instructions) for every join label of
    an exec-narrowing branch that runs vector work before restoring exec."""
    lines = text.splitlines()
    # join labels: targets of s_cbranch_execz that follow an exec-narrowing
    # instruction within the same basic block
    joins = set()
    narrowed = False
    for l in lines:
        t = l.strip()
        if _LABEL.match(t) or _FUNC.match(t):
            narrowed = False
            continue
        if _NARROW.match(t):
            narrowed = not _is_restore(t)
        m = _EXECZ.match(t)
        if m and narrowed:
            joins.add(m.group(1))
    found = []
    func = "?"
    for i, l in enumerate(lines):
        fm = _FUNC.match(l)
        if fm:
            func = fm.group(1)
            continue
        m = _LABEL.match(l)
        if not m or m.group(1) not in joins:
            continue
        extra = []
        for t in (x.strip() for x in lines[i + 1: i + 2000]):
            if not t or t.startswith(";"):
                continue
            if _is_restore(t):
                break
            if _NARROW.match(t) and not extra:
                break             # the block opens an else branch: its vector work has that branch's mask
            if _LABEL.match(t) or t.startswith(("s_cbranch", "s_branch", "s_endpgm", "s_setpc")):
                extra = []        # left the block without a restore: not this pattern
                break
            op = t.split()[0]
            if op.startswith(_VECTOR) and not op.startswith(_LANE_OPS):
                extra.append(t)
        if extra:
            found.append((func, i + 1, extra[:4]))
    return found


def check_files(paths) -> list[str]:
    """Human-readable findings over several assembly files."""
    out = []
    for p in paths:
        with open(p) as f:
            for func, line, extra in find_masked_joins(f.read()):
                out.append(f"{p}:{line}: {func}: vector work under a narrowed exec mask at a join: {extra}")
    return out


if __name__ == "__main__":
    problems = check_files(sys.argv[1:])
    print("\n".join(problems) if problems else "clean")
    sys.exit(1 if problems else 0)

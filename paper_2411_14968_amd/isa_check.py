"""Build-time check of the device code: no loop that holds a workgroup barrier may
also leave through a lane-divergent exit (`s_andn2_b64 exec, exec, ...`).

Such a loop means the compiler has restructured a barrier loop around a
lane-divergent branch; lanes then wait at the barrier for a lane that is held
outside the loop, and the workgroup never finishes. The check reads the
gfx950 assembly of the library's own sources.
"""
import collections
import re
import subprocess
import sys


def check_asm(txt: str) -> list[str]:
    funcs = re.findall(r"^(_Z\w+):.*?\n(.*?)s_endpgm", txt, flags=re.S | re.M)
    bad = []
    for name, body in funcs:
        cur = None
        blocks = collections.OrderedDict()
        for ln in body.split("\n"):
            m = re.match(r"^(\.LBB\w+|; %bb\.\d+):", ln)
            if m:
                cur = m.group(1)
                blocks[cur] = {"lines": [], "loop": None}
                if "This Loop Header" in ln:
                    blocks[cur]["loop"] = cur[2:] if cur.startswith(".L") else cur
                h = re.search(r"Header=(BB\w+) Depth=(\d+)", ln)
                if h:
                    blocks[cur]["loop"] = h.group(1)
                continue
            if cur:
                if "This Loop Header" in ln and blocks[cur]["loop"] is None:
                    blocks[cur]["loop"] = cur[2:] if cur.startswith(".L") else cur
                blocks[cur]["lines"].append(ln)
        loops = collections.defaultdict(list)
        for b, info in blocks.items():
            if info["loop"]:
                loops[info["loop"]].append(b)
        for hdr, members in loops.items():
            lines = [l for b in members for l in blocks[b]["lines"]]
            if any("s_barrier" in l for l in lines) and any(re.search(r"s_andn2_b64 exec, exec", l) for l in lines):
                bad.append(f"{name} (loop {hdr})")
    return bad


def check_sources(srcs: list[str], flags: list[str]) -> list[str]:
    bad = []
    for src in srcs:
        asm = subprocess.run(["hipcc", *flags, "--cuda-device-only", "-S", src, "-o", "-"],
                             check=True, capture_output=True, text=True).stdout
        bad += check_asm(asm)
    return bad


if __name__ == "__main__":
    found = check_asm(open(sys.argv[1]).read())
    print("\n".join(found) or "ok")
    sys.exit(1 if found else 0)

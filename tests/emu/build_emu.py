"""Build the library's device sources for the CPU emulation (hipemu) with
AddressSanitizer: a host shared library with the same C ABI as libsdgp.so.

The sources are copied with mechanical rewrites: kernel launches
`k<<<grid, block, shm, stream>>>(args)` become calls of the emulator's
launcher, the global address-space qualifier and the AMDGPU occupancy
attributes are dropped, and the context
workspace allocates exactly what each call asks for (no growth slack), so
that the sanitizer's bounds are the requested sizes.

    python tests/emu/build_emu.py [--src DIR] [--out LIB] [--include DIR] [--drop TEXT ...]
"""
from __future__ import annotations

import argparse
import glob
import os
import re
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CLANG = "/opt/rocm/llvm/bin/clang++"
CALLEE = re.compile(r"([A-Za-z_][\w:]*(?:<[^;{}()<>]*>)?)\s*$")


def _match_paren(s: str, i: int) -> int:
    """Index of the parenthesis closing the one at s[i]."""
    depth = 0
    for k in range(i, len(s)):
        if s[k] == "(":
            depth += 1
        elif s[k] == ")":
            depth -= 1
            if depth == 0:
                return k
    raise ValueError("unbalanced parentheses at %d" % i)


def rewrite_launches(src: str) -> str:
    out = []
    i = 0
    while True:
        j = src.find("<<<", i)
        if j < 0:
            out.append(src[i:])
            return "".join(out)
        m = CALLEE.search(src[i:j])
        if not m:
            raise ValueError("cannot find the kernel before <<< at %d" % j)
        callee = m.group(1)
        k = src.index(">>>", j)
        cfg = src[j + 3:k]
        a = k + 3
        while src[a].isspace():
            a += 1
        if src[a] != "(":
            raise ValueError("expected ( after >>> at %d" % a)
        b = _match_paren(src, a)
        args = src[a + 1:b].strip()
        out.append(src[i:i + m.start(1)])
        out.append('::emu::Cfg(%s).launch("%s", %s%s)' % (cfg, callee.replace('"', ""), callee,
                                                         (", " + args) if args else ""))
        i = b + 1


def drop_lines(text: str, drops, hits) -> str:
    """Remove the lines containing any of `drops` (a replay switches a
    guard off this way); hits counts the removed lines per pattern."""
    out = []
    for line in text.splitlines(keepends=True):
        d = [x for x in drops if x in line]
        for x in d:
            hits[x] += 1
        if not d:
            out.append(line)
    return "".join(out)


def rewrite(text: str) -> str:
    text = rewrite_launches(text)
    text = text.replace("__attribute__((address_space(1)))", "")
    text = re.sub(r"__attribute__\(\(amdgpu_[a-z_]+\([^()]*\)\)\)", "", text)
    text = text.replace('"../../include/sdgp.h"', '"sdgp.h"')
    text = re.sub(r"size_t cap = need \+ need / 8 \+ 256;", "size_t cap = need;", text)
    return text


def build(src_dir: str, out: str, jobs: int = 8, opt: str = "-O1", include: str = None, drops=(),
          defines=()) -> str:
    gen = out + ".src"
    os.makedirs(gen, exist_ok=True)
    include = include or os.path.join(ROOT, "include")
    hits = {x: 0 for x in drops}
    srcs = sorted(glob.glob(os.path.join(src_dir, "*.hip")) + glob.glob(os.path.join(src_dir, "*.cpp")))
    for h in glob.glob(os.path.join(src_dir, "*.hpp")):
        with open(h) as f, open(os.path.join(gen, os.path.basename(h)), "w") as g:
            g.write(rewrite(drop_lines(f.read(), drops, hits)))
    units = []
    for s in srcs:
        name = os.path.splitext(os.path.basename(s))[0] + ".cpp"
        with open(s) as f, open(os.path.join(gen, name), "w") as g:
            g.write(rewrite(drop_lines(f.read(), drops, hits)))
        units.append(os.path.join(gen, name))
    missing = [x for x, k in hits.items() if k == 0]
    if missing:
        raise RuntimeError("no source line contains %s" % missing)
    units.append(os.path.join(HERE, "hipemu.cpp"))
    flags = ["-std=c++17", opt, "-g", "-fPIC", "-fsanitize=address", "-shared-libsan", "-fno-omit-frame-pointer",
             "-Wno-unknown-attributes", "-Wno-unused-result", "-Wno-pass-failed",
             "-I", os.path.join(HERE, "include"), "-I", HERE, "-I", include, "-I", gen] + ["-D" + d for d in defines]

    def cc(u):
        o = os.path.join(gen, os.path.basename(u) + ".o")
        r = subprocess.run([CLANG] + flags + ["-c", u, "-o", o], capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("compile failed: %s\n%s" % (u, r.stderr[-6000:]))
        return o

    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(cc, units))
    r = subprocess.run([CLANG, "-shared", "-fsanitize=address", "-shared-libsan", "-o", out] + objs + ["-lpthread"],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s" % r.stderr[-4000:])
    return out


def asan_runtime() -> str:
    r = subprocess.run([CLANG, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    p = r.stdout.strip()
    if not os.path.exists(p):
        hits = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
        p = hits[0] if hits else p
    return p


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--src", default=os.path.join(ROOT, "paper_2205_09070_amd", "csrc"))
    ap.add_argument("--out", default=os.path.join(ROOT, "_build", "emu", "libsdgp_emu.so"))
    ap.add_argument("--opt", default="-O1")
    ap.add_argument("--include", default=None, help="directory of sdgp.h (default: the repository's)")
    ap.add_argument("--drop", action="append", default=[], help="remove source lines containing this text")
    ap.add_argument("--define", action="append", default=[], help="NAME=VALUE for the preprocessor")
    a = ap.parse_args()
    os.makedirs(os.path.dirname(a.out), exist_ok=True)
    print(build(a.src, a.out, opt=a.opt, include=a.include, drops=a.drop, defines=a.define))
    sys.exit(0)

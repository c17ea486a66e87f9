"""Builds the library's kernels and C ABI as host code under AddressSanitizer
and UndefinedBehaviorSanitizer.

    python tests/emu/build_emu.py          # -> tests/emu/libdpso_emu.so

Test infrastructure: the product sources are copied unchanged in meaning,
with these mechanical rewrites so that g++ compiles them against the
emulation header `tests/emu/include/hip/hip_runtime.h`:
  * kernel launches `k<<<grid, block, lds, stream>>>(args)` become
    `::emu::launch(k, grid, block, lds, stream, args)`;
  * the dynamic LDS declaration becomes a pointer to the workgroup's buffer;
  * address-space attributes, the scalar-register hint of `global_ptr` and the
    empty compiler fence (which becomes a wavefront synchronisation point) go;
  * `__builtin_amdgcn_*` becomes `emu_amdgcn_*` and the saturating add
    `emu_add_sat`;
  * a wavefront synchronisation point goes before every block that one lane
    of a wavefront runs alone (`if (lane == 0)` and the like): lanes of a
    wavefront execute in lockstep on the GPU, so every lane's earlier reads
    happen before that lane's writes, while the emulator runs lanes one after
    another between synchronisation points. Waves of a workgroup still run
    independently, as on the GPU.
The library is the one the GPU runs, less the voxel planner and viewpoint
selection; tests/emu/run_emu.py drives it (with the two sanitizer runtimes preloaded).
"""
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_1706_04399_amd", "csrc")
OUT = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libdpso_emu.so")
SOURCES = ["api.hip", "tune.hip", "swarm.hip", "twoopt.hip", "nodeswap.hip", "dist.hip", "checkdist.hip"]
HEADERS = ["device.hpp", "kernels.hpp", "state.hpp", "errors.hpp", "tune.hpp"]

LAUNCH = re.compile(r"(?P<k>[A-Za-z_][\w:]*(?:<[^<>;()]*>)?)<<<(?P<cfg>.+?)>>>\((?P<args>.*)\);")


def split_top(s):
    """Splits on commas outside parentheses, brackets and angle brackets."""
    out, depth, cur = [], 0, ""
    for ch in s:
        if ch in "([<":
            depth += 1
        elif ch in ")]>":
            depth -= 1
        if ch == "," and depth == 0:
            out.append(cur.strip())
            cur = ""
        else:
            cur += ch
    out.append(cur.strip())
    return out


def rewrite(text: str) -> str:
    def launch(m):
        cfg = split_top(m.group("cfg"))
        if len(cfg) != 4:
            raise ValueError(f"launch without 4 configuration arguments: {m.group(0)}")
        args = m.group("args").strip()
        return f"::emu::launch({m.group('k')}, {', '.join(cfg)}{', ' + args if args else ''});"

    n_launch = len(LAUNCH.findall(text))
    text = LAUNCH.sub(launch, text)
    assert "<<<" not in text, "a launch was not rewritten"
    text = text.replace("extern __shared__ __align__(16) unsigned char smem[];",
                        "unsigned char *smem = ::emu::dyn_lds();")
    text = re.sub(r"__attribute__\(\(address_space\(\d\)\)\)\s*", "", text)
    text = text.replace('__asm__("" : "+s"(g));', "")
    text = text.replace('__asm__ __volatile__("" ::: "memory");', "emu_wave_sync();")
    text = text.replace("__builtin_amdgcn_", "emu_amdgcn_")
    text = text.replace("__builtin_elementwise_add_sat", "emu_add_sat")
    text = re.sub(r"(?m)^(\s*)(if \((?:lane == 0|tid == 0|threadIdx\.x == 0|lane == 63|"
                  r"\(threadIdx\.x & 63\) == 0)\))", r"\1emu_wave_sync();\n\1\2", text)
    assert "__asm__" not in text, "inline asm left in the emulated sources"
    return text, n_launch


def _up_to_date() -> bool:
    """The library is newer than every source it is built from."""
    if not os.path.exists(LIB):
        return False
    t = os.path.getmtime(LIB)
    deps = [os.path.join(CSRC, f) for f in HEADERS + SOURCES] + [os.path.join(HERE, "emu.cpp"), __file__,
            os.path.join(HERE, "include", "hip", "hip_runtime.h"), os.path.join(ROOT, "include", "dpso.h")]
    return all(os.path.getmtime(d) < t for d in deps)


def build(verbose=True) -> str:
    """Builds the library unless it is up to date. Concurrent callers (test
    workers) take turns on a lock file, and the library is replaced in one
    step, so a reader never sees a partial file."""
    import fcntl
    os.makedirs(OUT, exist_ok=True)
    with open(os.path.join(OUT, ".lock"), "w") as lock:
        fcntl.flock(lock, fcntl.LOCK_EX)
        if _up_to_date():
            return LIB
        return _build(verbose)


def _build(verbose) -> str:
    objs, launches = [], 0
    for name in HEADERS + SOURCES:
        text, n = rewrite(open(os.path.join(CSRC, name)).read())
        launches += n
        dst = os.path.join(OUT, name.replace(".hip", ".cpp"))
        with open(dst, "w") as f:
            f.write(text)
    flags = ["-std=c++17", "-O1", "-g", "-fPIC", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
             "-Wno-attributes", "-Wno-ignored-attributes", "-Wno-unused-result",
             "-I", os.path.join(HERE, "include"), "-I", os.path.join(ROOT, "include"), "-I", OUT]
    srcs = [os.path.join(OUT, s.replace(".hip", ".cpp")) for s in SOURCES] + [os.path.join(HERE, "emu.cpp")]
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = ["g++"] + flags + ["-shared", "-o", tmp] + srcs
    if verbose:
        print(" ".join(cmd), flush=True)
        print(f"{launches} kernel launches rewritten", flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stderr[-20000:])
        raise RuntimeError("host build of the emulated library failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())

"""Builds the CPU-executor driver (library sources + simt runtime) with
AddressSanitizer -- TEST INFRASTRUCTURE ONLY.  Output:
tests/simt_cpu/_build/wr_cpu_driver."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2504_20655_amd", "csrc")
OUT = os.path.join(HERE, "_build", "wr_cpu_driver")
LIB_SOURCES = ["kernels.hip", "runtime.cpp", "tiles.cpp", "solve.cpp", "server.cpp", "autotune.cpp",
               "routes.cpp", "wms.hip"]


def build(sanitize: bool = True) -> str:
    """Compiles into a directory of this process and renames the linked
    driver into place, so parallel test workers never write a file another
    one is running or linking."""
    import shutil
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    objdir = os.path.join(os.path.dirname(OUT), f"obj{os.getpid()}")
    os.makedirs(objdir, exist_ok=True)
    san = ["-fsanitize=address", "-fno-omit-frame-pointer"] if sanitize else []
    flags = ["-std=c++20", "-O1", "-g", "-pthread", "-w", *san,
             "-I", HERE, "-I", os.path.join(ROOT, "include")]
    objs = []
    procs = []
    for src in LIB_SOURCES + ["../../tests/simt_cpu/simt_runtime.cpp", "../../tests/simt_cpu/driver.cpp"]:
        path = os.path.normpath(os.path.join(CSRC, src))
        if not os.path.exists(path):
            continue
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        cmd = ["g++", "-x", "c++", *flags, "-c", path, "-o", obj]
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
        objs.append(obj)
    for src, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            raise RuntimeError(f"{src}:\n{out}")
    tmp = f"{OUT}.tmp{os.getpid()}"
    r = subprocess.run(["g++", *san, "-pthread", "-o", tmp, *objs], capture_output=True, text=True)
    shutil.rmtree(objdir, ignore_errors=True)
    if r.returncode != 0:
        raise RuntimeError(r.stdout + r.stderr)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(sanitize="--no-asan" not in sys.argv))

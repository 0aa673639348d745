"""Build libfcfs's kernels and host code for the CPU under the host emulation
(test infrastructure; see hip/hip_runtime.h), with the address sanitizer."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2203_10670_amd", "csrc")
# extra -D flags (compile-time tuning switches of the kernels) build a separate library
EXTRA = os.environ.get("FCFS_HOSTEMU_DEFINES", "").split()
OUT = os.path.join(HERE, "_build", "libfcfs_hostemu%s.so" % ("_" + "_".join(d.lstrip("-D") for d in EXTRA) if EXTRA
                                                            else ""))
SOURCES = ["api.cpp", "fwd_plan.cpp", "fwd_f32.hip", "fwd_bf16.hip", "fwd_f16.hip", "bwd_f32.hip", "bwd_bf16.hip", "bwd_f16.hip", "bwd_mix.hip",
           "mix4.hip", "mix4_f32.hip"]
CXX = "/opt/rocm/llvm/bin/clang++"   # host compile; knows __bf16, _Float16 and vector extensions


def build(sanitize: bool = True) -> str:
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    srcs = [os.path.join(CSRC, s) for s in SOURCES] + [os.path.join(HERE, "emu_main.cpp")]
    newest = max(os.path.getmtime(s) for s in srcs + [os.path.join(HERE, "hip", "hip_runtime.h"), __file__,
                                                       os.path.join(CSRC, "fcfs_internal.h")] +
                 [os.path.join(CSRC, h) for h in os.listdir(CSRC) if h.endswith(".h")])
    if os.path.exists(OUT) and os.path.getmtime(OUT) >= newest:
        return OUT
    flags = ["-std=c++20", "-O2", "-g", "-fPIC", "-shared", "-pthread", "-w",
             "-I", HERE, "-I", os.path.join(ROOT, "include"), "-I", CSRC] + EXTRA
    if sanitize:
        flags += ["-fsanitize=address,undefined", "-fno-omit-frame-pointer"]
    from concurrent.futures import ThreadPoolExecutor
    objdir = os.path.join(os.path.dirname(OUT), "obj" + ("_" + "_".join(d.lstrip("-D") for d in EXTRA) if EXTRA
                                                         else ""))
    os.makedirs(objdir, exist_ok=True)

    def compile_one(src):
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        subprocess.check_call([CXX] + [f for f in flags if f != "-shared"] + ["-c", "-x", "c++", src, "-o", obj])
        return obj

    with ThreadPoolExecutor(max(1, min(len(srcs), os.cpu_count() or 2))) as ex:
        objs = list(ex.map(compile_one, srcs))
    tmp = OUT + ".tmp%d" % os.getpid()
    subprocess.check_call([CXX] + flags + ["-shared-libsan"] + objs + ["-o", tmp])
    os.replace(tmp, OUT)
    return OUT


def asan_runtime() -> str:
    return subprocess.check_output([CXX, "-print-file-name=libclang_rt.asan-x86_64.so"], text=True).strip()


if __name__ == "__main__":
    print(build())

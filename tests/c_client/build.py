"""Build the C++ ABI client used by tests/test_zz_c_client.py (host code only,
linked against the library's libcorr.so with a relative rpath)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
LIBDIR = os.path.join(ROOT, "paper_1305_5639_amd")
OUT = os.path.join(HERE, "corr_client")


def build() -> str:
    cmd = ["/opt/rocm/bin/hipcc", "-O2", "-std=c++17", "--offload-arch=gfx950",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           f"-I{os.path.join(ROOT, 'include')}", os.path.join(HERE, "corr_client.cpp"),
           f"-L{LIBDIR}", "-lcorr", "-Wl,-rpath,$ORIGIN/../../paper_1305_5639_amd", "-o", OUT + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("corr_client build failed:\n" + r.stdout + r.stderr)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    print(build())

"""Build helper of the plain C client of the C ABI (tests/c/gmf_c_client.c):
gcc against include/gmf.h and the in-tree libgmf.so, nothing else."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "c", "gmf_c_client.c")
EXE = os.path.join(ROOT, "tests", "c", "gmf_c_client")
LIBDIR = os.path.join(ROOT, "paper_2601_03806_amd")


def build(force: bool = False) -> str:
    """Compile the client unless an up-to-date binary is there."""
    lib = os.path.join(LIBDIR, "libgmf.so")
    if not os.path.exists(lib):
        raise FileNotFoundError(f"{lib} is missing: build the HIP library first")
    if (not force and os.path.exists(EXE) and os.path.getmtime(EXE) >= os.path.getmtime(SRC)
            and os.path.getmtime(EXE) >= os.path.getmtime(lib)):
        return EXE
    tmp = EXE + ".tmp"
    subprocess.run(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-Werror", f"-I{os.path.join(ROOT, 'include')}",
                    SRC, "-o", tmp, f"-L{LIBDIR}", "-lgmf", f"-Wl,-rpath,{LIBDIR}", "-lm"], check=True)
    os.replace(tmp, EXE)
    return EXE

"""The binding imports torch before it loads the library, so both use one HIP runtime
(torch ships its own under the same soname); checked in a fresh interpreter on the CPU."""
import ast
import subprocess
import sys
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_binding_loads_torch_before_the_library():
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2412_17510_amd import mp\n"
            "import torch, os\n"
            "maps = open('/proc/self/maps').read().splitlines()\n"
            "libs = [l.split()[-1] for l in maps if 'libamdhip64' in l]\n"
            "print(sorted(set(libs)))\n" % ROOT)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    libs = ast.literal_eval(out.stdout.strip().splitlines()[-1])
    torch_dir = os.path.dirname(__import__("torch").__file__)
    assert len(libs) == 1 and libs[0].startswith(torch_dir), libs

"""The examples of README.md: the C program built against include/oif.h and
liboif.so, the Python program's source."""
import os
import re
import shutil
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def build_readme_example(out_dir) -> str:
    """Extract the C program that follows the `example.c` marker in README.md,
    compile and link it with gcc; returns the executable's path."""
    gcc = shutil.which("gcc")
    if gcc is None:
        raise FileNotFoundError("gcc not available")
    text = open(os.path.join(ROOT, "README.md")).read()
    m = re.search(r"<!-- example.c -->\n```c\n(.*?)```", text, re.S)
    assert m, "README.md holds no C example"
    src = os.path.join(str(out_dir), "example.c")
    exe = os.path.join(str(out_dir), "example")
    with open(src, "w") as fh:
        fh.write(m.group(1))
    lib_dir = os.path.join(ROOT, "paper_1312_3426_amd")
    subprocess.run([gcc, "-Wall", "-Wextra", "-Werror", "-I" + os.path.join(ROOT, "include"), src,
                    "-L" + lib_dir, "-loif", "-Wl,-rpath," + lib_dir, "-o", exe], check=True,
                   capture_output=True, text=True)
    return exe


def readme_python_example() -> str:
    """The Python program that follows the `example.py` marker in README.md."""
    text = open(os.path.join(ROOT, "README.md")).read()
    m = re.search(r"<!-- example.py -->\n```python\n(.*?)```", text, re.S)
    assert m, "README.md holds no Python example"
    return m.group(1)

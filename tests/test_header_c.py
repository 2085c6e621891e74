"""include/su3.h is a C header: a C11 translation unit that includes it and
takes the address of every declared entry point compiles cleanly with gcc
-Wall -Wextra -Werror -pedantic (no HIP headers needed, streams are void *)."""

import os
import re
import subprocess
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "su3.h")


def test_header_compiles_as_c11():
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    names = sorted(set(re.findall(r"\b(su3_[a-z0-9_]+)\s*\(", text)))
    assert len(names) >= 12
    body = ['#include "su3.h"', "#include <stdio.h>", "int main(void) {", "    void *fns[] = {"]
    body += ["        (void *)(size_t)&%s," % n for n in names]
    body += ["    };", '    printf("%d %d\\n", (int)(sizeof fns / sizeof fns[0]), SU3_ABI_VERSION);',
             "    return SU3_OK + SU3_F64;", "}"]
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "t.c")
        open(src, "w").write("\n".join(body) + "\n")
        proc = subprocess.run(["gcc", "-std=c11", "-Wall", "-Wextra", "-Werror", "-pedantic", "-I",
                               os.path.join(ROOT, "include"), "-c", src, "-o", os.path.join(d, "t.o")],
                              capture_output=True, text=True)
        assert proc.returncode == 0, proc.stderr

"""Hash of the kernel sources, used to tie measured profile figures to the
exact kernel version they were taken on."""
import hashlib
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
SOURCES = [os.path.join(_PKG, "csrc", "gray.hip"), os.path.join(_PKG, "csrc", "kerr.hpp"),
           os.path.join(os.path.dirname(_PKG), "include", "gray.h")]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    print(kernel_source_hash())

"""Hash of the HIP sources, used to tell whether recorded hardware-counter
measurements still describe the current kernels."""
import hashlib
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(HERE, "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    print(source_hash())

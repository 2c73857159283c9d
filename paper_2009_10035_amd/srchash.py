"""Hash of the sources of the update kernel (its template, the device helpers
and argument structs it includes, its instance files, and the host code that
chooses its launch and work-unit parameters), used to tell whether recorded
hardware-counter measurements still describe it."""
import hashlib
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(HERE, "csrc")
    names = [x for x in os.listdir(csrc)
             if x in ("f2v_device.h", "f2v_kernels.h", "f2v_update_impl.h", "f2v_api.cpp")
             or x.startswith("f2v_variants")]
    for name in sorted(names):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    print(source_hash())

"""Build and run the operation counter (csrc/opcount.cpp) and store its
result in opcount.json, which the benchmark uses for algorithmic flops."""
import json
import os
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "opcount.json")


def run():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "opcount")
        subprocess.run(["hipcc", "-x", "hip", "-std=c++20", "-O1", "--offload-arch=gfx950", "-o", exe,
                        os.path.join(HERE, "csrc", "opcount.cpp")], check=True)
        res = json.loads(subprocess.run([exe], check=True, capture_output=True, text=True).stdout)
    with open(OUT, "w") as f:
        json.dump(res, f, indent=1)
    return res


if __name__ == "__main__":
    print(json.dumps(run(), indent=1))

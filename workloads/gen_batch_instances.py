"""Write the batched-workload instance table (numpy PCG64, seed 2024) to JSON."""
import json
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import workloads  # noqa: E402

if __name__ == "__main__":
    inst = workloads.generate_batch_instances()
    with open(workloads.BATCH_JSON, "w") as f:
        f.write("[\n" + ",\n".join(json.dumps(i, separators=(",", ":")) for i in inst) + "\n]\n")
    tot = sum(i["paths"] for i in inst)
    print(f"wrote {len(inst)} instances, {tot} paths total to {workloads.BATCH_JSON}")

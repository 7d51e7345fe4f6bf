"""Host logic of bench.py: the counter summaries under profiles/ are used
only for the kernel sources and step window they were taken on."""
import os

import bench


def _write(root, name, kv):
    d = os.path.join(root, "profiles")
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, name), "w") as fh:
        fh.write("# summary\n" + "".join(f"{k}: {v}\n" for k, v in kv.items()))


def test_counter_summaries_guarded(tmp_path, monkeypatch):
    """A summary with another digest or window gives None; the right one its value."""
    digest = bench.kernel_digest()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_digest", lambda: digest)
    w = "gold_512cube_2e8_fp32"
    assert bench.counted_traffic(w, (105, 125)) is None and bench.counted_valu(w, (105, 125)) is None
    _write(str(tmp_path), f"particle_kernel_hbm_bytes_{w}.txt",
           {"kernel_digest": digest, "window": "105-125", "hbm_bytes_per_launch": "123456"})
    _write(str(tmp_path), f"particle_kernel_valu_{w}.txt",
           {"kernel_digest": digest, "window": "105-125", "valu_insts_per_launch": "789"})
    assert bench.counted_traffic(w, (105, 125)) == 123456
    assert bench.counted_valu(w, (105, 125)) == 789.0
    assert bench.counted_traffic(w, (55, 75)) is None and bench.counted_valu(w, (55, 75)) is None
    monkeypatch.setattr(bench, "kernel_digest", lambda: "0" * 16)
    assert bench.counted_traffic(w, (105, 125)) is None and bench.counted_valu(w, (105, 125)) is None


def test_digest_ignores_comments(tmp_path, monkeypatch):
    """Comments and blank lines do not move the digest; code does."""
    src = tmp_path / "a.hip"
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "KERNEL_SOURCES", ("a.hip",))
    src.write_text("int f(int x) {\n  return x + 1;\n}\n")
    d0 = bench.kernel_digest()
    src.write_text("// header\nint f(int x) {  // the step\n\n  /* one */return x + 1;\n}\n")
    assert bench.kernel_digest() == d0
    src.write_text("int f(int x) {\n  return x + 2;\n}\n")
    assert bench.kernel_digest() != d0

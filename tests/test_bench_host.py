"""Host-side logic of bench.py (no GPU needed): the counter traffic it reports
comes from the committed summaries only while the kernel source they were
taken on is unchanged, and only for the tag of the measured configuration."""
import bench


def write_summary(path, tag, digest, nbytes):
    with open(path, "w") as f:
        f.write("# summary\n\nsome text\n\n")
        f.write(f"    traffic {tag} {digest} {nbytes}\n")


def test_traffic_needs_matching_tag_and_source(tmp_path):
    src = tmp_path / "kernel.hip"
    src.write_text("kernel source, first version\n")
    summary = tmp_path / "summary.md"
    write_summary(summary, "step64_c2_1024", bench.source_digest(str(src)), 622503674)
    assert bench.committed_traffic("step64_c2_1024", str(summary), str(src)) == 622503674.0
    # another configuration's tag is not reported
    assert bench.committed_traffic("step64_c2_2048", str(summary), str(src)) is None
    # an edited source voids the figure
    src.write_text("kernel source, second version\n")
    assert bench.committed_traffic("step64_c2_1024", str(summary), str(src)) is None
    # a missing summary reports nothing
    assert bench.committed_traffic("step64_c2_1024", str(tmp_path / "none.md"), str(src)) is None


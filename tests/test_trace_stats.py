"""The trace summariser splits a kernel trace into searches by their
dedispersion launches."""
import os

from paper_1802_03084_amd import trace_stats


def test_searches_split_by_dedispersion_launches(tmp_path):
    p = os.path.join(tmp_path, "t.csv")
    with open(p, "w") as f:
        f.write("Kernel_Name,Start_Timestamp,End_Timestamp\n")
        f.write('"void (anonymous namespace)::k_drs<float2, 2>(x)",0,1000\n')
        f.write('"void (anonymous namespace)::k_cols_stats<1024>(x)",1000,3000\n')
        f.write('"void (anonymous namespace)::k_cols_stats<1024>(x)",3000,4000\n')
        f.write('"void (anonymous namespace)::k_drs<float2, 2>(x)",5000,6000\n')
        f.write('"void (anonymous namespace)::k_cols_stats<1024>(x)",6000,7000\n')
        f.write('"void at::native::other(x)",7000,9000\n')
    s = trace_stats.searches(p, 1)
    assert len(s) == 2
    assert s[0][1]["k_cols_stats"] == (1.5, 2) and s[1][1]["k_cols_stats"] == (1.0, 1)
    assert abs(s[0][0] - 0.004) < 1e-12

"""Host logic of the request server (no GPU)."""
from paper_2607_05622_amd import serve


def test_graph_buckets_follow_digestion_groups():
    # up to 8 densities one group of 8, beyond that groups of 16: a request
    # replays the graph of its own group count, never one with an extra group
    assert serve._buckets(64) == [8, 16, 32, 48, 64]
    assert serve._buckets(8) == [8]
    for nd in range(1, 65):
        b = serve._bucket(nd)
        assert b >= nd and b in serve._buckets(64)
        groups = lambda k: 1 if k <= 8 else (k + 15) // 16
        assert groups(b) == groups(nd)

"""CPU checks of the serving loop's host logic: which requests take the HSMG
pressure preconditioner and how that splits the batch keys (no GPU needed)."""
from paper_2608_24348_amd import inputs, serve


def _spec(N, nel, kind="tgv", tier="fp32b"):
    return {"N": N, "nel": nel, "kind": kind, "tier": tier}


def test_hsmg_eligibility_follows_the_library_limits():
    # order >= 4 and 2..64 elements per direction (the limits sem_setup enforces)
    assert serve._hsmg_ok(_spec(5, (4, 4, 4)))
    assert serve._hsmg_ok(_spec(4, (2, 64, 2)))
    assert not serve._hsmg_ok(_spec(3, (4, 4, 4)))
    assert not serve._hsmg_ok(_spec(7, (1, 4, 4)))
    assert not serve._hsmg_ok(_spec(7, (4, 65, 4)))


def test_batch_key_carries_the_preconditioner():
    a = serve._key(_spec(5, (4, 4, 4)), hsmg=1)
    b = serve._key(_spec(5, (4, 4, 4)), hsmg=0)
    c = serve._key(_spec(3, (4, 4, 4)), hsmg=1)       # not eligible: Jacobi
    assert a[:3] == b[:3] and a[3] == 1 and b[3] == 0
    assert c[3] == 0 and c[2] == "tgv"
    # requests of one key share order, tier, kind and preconditioner, so a
    # batch is always valid for the library (same lx, policy and hsmg flag)
    specs = inputs.request_stream(n_requests=64, qps=10.0, seed=5, nmin=1, nmax=6, orders=(3, 5))
    keys = {}
    for s in specs:
        r = serve.Request(s, 1)
        keys.setdefault(r.key, []).append(s)
    for k, group in keys.items():
        assert all(g["N"] + 1 == k[0] and g["tier"] == k[1] and g["kind"] == k[2] for g in group)
        assert all(serve._hsmg_ok(g) == bool(k[3]) for g in group)
    assert any(k[3] == 1 for k in keys) and any(k[3] == 0 for k in keys)

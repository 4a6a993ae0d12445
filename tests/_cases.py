"""Shared test helpers: one description of a filter, turned into the
library's configuration and the oracle's configuration independently."""
import numpy as np

LL_PARAMS = dict(x0_mean=0.0, x0_var=10.0, sigma_v2=1.0, sigma_w2=0.1)
LL_PL_PARAMS = dict(x0_mean=0.0, x0_var=10.0, a_v=2.0, b_v=1.0, a_w=2.0, b_w=1.0)
MU, PHI, SIG = -1.0, 0.95, 0.2
SV_X0 = dict(x0_mean=MU, x0_var=SIG**2 / (1 - PHI**2))
SV_PF_PARAMS = dict(SV_X0, mu=MU, phi=PHI, sigma2=SIG**2)
SV_PL_PARAMS = dict(SV_X0, prior_mean=[MU * (1 - PHI), PHI], prior_prec=[1.0, 0.0, 1.0],
                    a_s=2.0, d_s=0.04)
PARAMS = {"ll_pf": LL_PARAMS, "ll_pl": LL_PL_PARAMS, "sv_pf": SV_PF_PARAMS,
          "sv_pl": SV_PL_PARAMS}
MODEL_ID = {"ll_pf": 0, "ll_pl": 1, "sv_pf": 2, "sv_pl": 3}
SCHEME_ID = {"multinomial": 0, "stratified": 1, "systematic": 2, "sorted_multinomial": 3}


def data(model, T, seed=0):
    from paper_1212_1639_amd import inputs
    if model.startswith("ll"):
        return inputs.local_level(T, seed=seed)[0]
    return inputs.stochastic_volatility(T, seed=seed)[0]


def oracle_config(orc, model, n, seed, scheme, fp32):
    return orc.make_config(MODEL_ID[model], n, seed, scheme=SCHEME_ID[scheme],
                           fp32_words=fp32, **PARAMS[model])


def pf_config(pf, model, n, seed, scheme, fp32, strategy=0, ipt=0, keep_ancestors=True,
              lookback=False):
    flags = (pf.FLAG_KEEP_ANCESTORS if keep_ancestors else 0) | (
        pf.FLAG_LOOKBACK_SCAN if lookback else 0)
    return pf.make_config(MODEL_ID[model], n, seed, scheme=SCHEME_ID[scheme],
                          precision=pf.FP32 if fp32 else pf.FP64, strategy=strategy,
                          items_per_thread=ipt, flags=flags, **PARAMS[model])


def oracle_to_record(orc, model, ocfg, state):
    """Oracle state (F_oracle, N) -> the library's record fields (F, N)."""
    if model != "sv_pl":
        return state
    p = PARAMS[model]
    P0, P1, P2 = p["prior_prec"]
    b0a, b0b = p["prior_mean"]
    eta0a, eta0b = P0 * b0a + P1 * b0b, P1 * b0a + P2 * b0b
    x, n, S1, S11, Sy, S1y, Syy = state
    d = np.array([orc.sv_posterior(ocfg, [n[i], S1[i], S11[i], Sy[i], S1y[i], Syy[i]])[6]
                  for i in range(x.size)])
    return np.stack([x, P1 + S1, P2 + S11, eta0a + Sy, eta0b + S1y, d])


def record_to_oracle(model, rec, t0):
    """The library's record (F, N) after t0 steps -> oracle fields (F_oracle, N)."""
    rec = np.asarray(rec, dtype=np.float64)
    if model != "sv_pl":
        return rec
    p = PARAMS[model]
    P0, P1, P2 = p["prior_prec"]
    b0a, b0b = p["prior_mean"]
    eta0a, eta0b = P0 * b0a + P1 * b0b, P1 * b0a + P2 * b0b
    quad0 = b0a * eta0a + b0b * eta0b
    x, L01, L11, e0, e1, d = rec
    L00 = P0 + t0
    det = L00 * L11 - L01 * L01
    m0 = (L11 * e0 - L01 * e1) / det
    m1 = (L00 * e1 - L01 * e0) / det
    mlm = m0 * e0 + m1 * e1  # m' Lambda m = eta' Lambda^{-1} eta
    Syy = 2.0 * (d - p["d_s"]) - quad0 + mlm
    n = np.full_like(x, float(t0))
    return np.stack([x, n, L01 - P1, L11 - P2, e0 - eta0a, e1 - eta0b, Syy])

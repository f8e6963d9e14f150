// Table of the binary64 log2 in vnp_nodes_p.hpp, written by lp_coeffs.py (do not edit).
// Entry j (the top 7 fraction bits of v in [1/2, 1)): {c_j, l_j} with
// c_j = RN(1 / mid_j), mid_j = 1/2 + (j + 1/2) / 256, and l_j = RN(log2(2 / c_j)).
// Power table (Z^(1/p) for Z in [1, 2)): entry j (the top 7 fraction bits of Z)
// is c'_j = RN(128 / (128 + j)), the reciprocal of the interval's left end.
#pragma once

namespace vnp {

constexpr int LP_TAB_BITS = 7;
#define VNP_LP_LOG_TAB \
    { \
        {0x1.fe01fe01fe020p+0, 0x1.709c46d7aac60p-8}, \
        {0x1.fa11caa01fa12p+0, 0x1.1363117a97b03p-6}, \
        {0x1.f6310aca0dbb5p+0, 0x1.c9363ba850f9cp-6}, \
        {0x1.f25f644230ab5p+0, 0x1.3ed3094685a27p-5}, \
        {0x1.ee9c7f8458e02p+0, 0x1.985bfc3495193p-5}, \
        {0x1.eae807aba01ebp+0, 0x1.f13898332539dp-5}, \
        {0x1.e741aa59750e4p+0, 0x1.24b5b7e135a41p-4}, \
        {0x1.e3a9179dc1a73p+0, 0x1.507b836033bbap-4}, \
        {0x1.e01e01e01e01ep+0, 0x1.7beee96b8a281p-4}, \
        {0x1.dca01dca01dcap+0, 0x1.a7111df348494p-4}, \
        {0x1.d92f2231e7f8ap+0, 0x1.d1e34e35b82d7p-4}, \
        {0x1.d5cac807572b2p+0, 0x1.fc66a0f0b00a5p-4}, \
        {0x1.d272ca3fc5b1ap+0, 0x1.134e1b4890631p-3}, \
        {0x1.cf26e5c44bfc6p+0, 0x1.284294b07a640p-3}, \
        {0x1.cbe6d9601cbe7p+0, 0x1.3d1146d9a8a63p-3}, \
        {0x1.c8b265afb8a42p+0, 0x1.51bab907a5c8ap-3}, \
        {0x1.c5894d10d4986p+0, 0x1.663f6fac91315p-3}, \
        {0x1.c26b5392ea01cp+0, 0x1.7a9fec7d05de0p-3}, \
        {0x1.bf583ee868d8bp+0, 0x1.8edcae8352b6bp-3}, \
        {0x1.bc4fd65883e7bp+0, 0x1.a2f632320b86cp-3}, \
        {0x1.b951e2b18ff23p+0, 0x1.b6ecf175f95ecp-3}, \
        {0x1.b65e2e3beee05p+0, 0x1.cac163c770dcap-3}, \
        {0x1.b37484ad806cep+0, 0x1.de73fe3b1480ep-3}, \
        {0x1.b094b31d922a4p+0, 0x1.f205339208f27p-3}, \
        {0x1.adbe87f94905ep+0, 0x1.02baba24d0664p-2}, \
        {0x1.aaf1d2f87ebfdp+0, 0x1.0c62975542a8dp-2}, \
        {0x1.a82e65130e159p+0, 0x1.15fa676bb08fep-2}, \
        {0x1.a574107688a4ap+0, 0x1.1f825f6d88e13p-2}, \
        {0x1.a2c2a87c51ca0p+0, 0x1.28fab35b32684p-2}, \
        {0x1.a01a01a01a01ap+0, 0x1.32639636b2836p-2}, \
        {0x1.9d79f176b682dp+0, 0x1.3bbd3a0a1dcfbp-2}, \
        {0x1.9ae24ea5510dap+0, 0x1.4507cfedd4fc5p-2}, \
        {0x1.9852f0d8ec0ffp+0, 0x1.4e43880e8fb6bp-2}, \
        {0x1.95cbb0be377aep+0, 0x1.577091b3378c9p-2}, \
        {0x1.934c67f9b2ce6p+0, 0x1.608f1b42948aep-2}, \
        {0x1.90d4f120190d5p+0, 0x1.699f5248cd4b8p-2}, \
        {0x1.8e6527af1373fp+0, 0x1.72a1637cbc183p-2}, \
        {0x1.8bfce8062ff3ap+0, 0x1.7b957ac51aac4p-2}, \
        {0x1.899c0f601899cp+0, 0x1.847bc33d8618ep-2}, \
        {0x1.87427bcc092b9p+0, 0x1.8d54673b5c371p-2}, \
        {0x1.84f00c2780614p+0, 0x1.961f90527409bp-2}, \
        {0x1.82a4a0182a4a0p+0, 0x1.9edd6759b25e0p-2}, \
        {0x1.8060180601806p+0, 0x1.a78e146f7bef4p-2}, \
        {0x1.7e225515a4f1dp+0, 0x1.b031befe06435p-2}, \
        {0x1.7beb3922e017cp+0, 0x1.b8c88dbf88679p-2}, \
        {0x1.79baa6bb6398bp+0, 0x1.c152a6c24cae7p-2}, \
        {0x1.77908119ac60dp+0, 0x1.c9d02f6ca47b5p-2}, \
        {0x1.756cac201756dp+0, 0x1.d2414c80bf27cp-2}, \
        {0x1.734f0c541fe8dp+0, 0x1.daa6222064fb8p-2}, \
        {0x1.713786d9c7c09p+0, 0x1.e2fed3d097297p-2}, \
        {0x1.6f26016f26017p+0, 0x1.eb4b847d15bcep-2}, \
        {0x1.6d1a62681c861p+0, 0x1.f38c567bcc541p-2}, \
        {0x1.6b1490aa31a3dp+0, 0x1.fbc16b902680ap-2}, \
        {0x1.691473a88d0c0p+0, 0x1.01f57277264e0p-1}, \
        {0x1.6719f3601671ap+0, 0x1.0604719f24eb2p-1}, \
        {0x1.6524f853b4aa3p+0, 0x1.0a0dc34f8e1fcp-1}, \
        {0x1.63356b88ac0dep+0, 0x1.0e117754d7c11p-1}, \
        {0x1.614b36831ae94p+0, 0x1.120f9d39e1806p-1}, \
        {0x1.5f66434292dfcp+0, 0x1.160844495e006p-1}, \
        {0x1.5d867c3ece2a5p+0, 0x1.19fb7b8f32422p-1}, \
        {0x1.5babcc647fa91p+0, 0x1.1de951d9cbba7p-1}, \
        {0x1.59d61f123ccaap+0, 0x1.21d1d5bb6d59bp-1}, \
        {0x1.5805601580560p+0, 0x1.25b5158b73d05p-1}, \
        {0x1.56397ba7c52e2p+0, 0x1.29931f6791560p-1}, \
        {0x1.54725e6bb82fep+0, 0x1.2d6c013501380p-1}, \
        {0x1.52aff56a8054bp+0, 0x1.313fc8a1b36f2p-1}, \
        {0x1.50f22e111c4c5p+0, 0x1.350e8325707dap-1}, \
        {0x1.4f38f62dd4c9bp+0, 0x1.38d83e02f5d08p-1}, \
        {0x1.4d843bedc2c4cp+0, 0x1.3c9d06490ae11p-1}, \
        {0x1.4bd3edda68fe1p+0, 0x1.405ce8d38f4bcp-1}, \
        {0x1.4a27fad76014ap+0, 0x1.4417f24c82165p-1}, \
        {0x1.4880522014880p+0, 0x1.47ce2f2d02588p-1}, \
        {0x1.46dce34596066p+0, 0x1.4b7fabbe49796p-1}, \
        {0x1.453d9e2c776cap+0, 0x1.4f2c741a9f33ep-1}, \
        {0x1.43a2730abee4dp+0, 0x1.52d4942e4790ap-1}, \
        {0x1.420b5265e5951p+0, 0x1.567817b86b02dp-1}, \
        {0x1.40782d10e6566p+0, 0x1.5a170a4bf8d5cp-1}, \
        {0x1.3ee8f42a5af07p+0, 0x1.5db177508413cp-1}, \
        {0x1.3d5d991aa75c6p+0, 0x1.61476a031b108p-1}, \
        {0x1.3bd60d9232955p+0, 0x1.64d8ed7719beep-1}, \
        {0x1.3a524387ac822p+0, 0x1.68660c96f6f88p-1}, \
        {0x1.38d22d366088ep+0, 0x1.6beed2250cdadp-1}, \
        {0x1.3755bd1c945eep+0, 0x1.6f7348bc5c617p-1}, \
        {0x1.35dce5f9f2af8p+0, 0x1.72f37ad14c5b0p-1}, \
        {0x1.34679ace01346p+0, 0x1.766f72b263defp-1}, \
        {0x1.32f5ced6a1dfap+0, 0x1.79e73a8900620p-1}, \
        {0x1.3187758e9ebb6p+0, 0x1.7d5adc5a078a4p-1}, \
        {0x1.301c82ac40260p+0, 0x1.80ca620694df9p-1}, \
        {0x1.2eb4ea1fed14bp+0, 0x1.8435d54ca3774p-1}, \
        {0x1.2d50a012d50a0p+0, 0x1.879d3fc7b3b71p-1}, \
        {0x1.2bef98e5a3711p+0, 0x1.8b00aaf16d4a9p-1}, \
        {0x1.2a91c92f3c105p+0, 0x1.8e6020223d661p-1}, \
        {0x1.293725bb804a5p+0, 0x1.91bba891f1708p-1}, \
        {0x1.27dfa38a1ce4dp+0, 0x1.95134d584e2e4p-1}, \
        {0x1.268b37cd60127p+0, 0x1.9867176da382dp-1}, \
        {0x1.2539d7e9177b2p+0, 0x1.9bb70fab5ce4dp-1}, \
        {0x1.23eb79717605bp+0, 0x1.9f033ecc8e957p-1}, \
        {0x1.22a0122a0122ap+0, 0x1.a24bad6e7fb77p-1}, \
        {0x1.21579804855e6p+0, 0x1.a590641131564p-1}, \
        {0x1.2012012012012p+0, 0x1.a8d16b17e2745p-1}, \
        {0x1.1ecf43c7fb84cp+0, 0x1.ac0ecac99133cp-1}, \
        {0x1.1d8f5672e4abdp+0, 0x1.af488b51792d4p-1}, \
        {0x1.1c522fc1ce059p+0, 0x1.b27eb4bf8f08ap-1}, \
        {0x1.1b17c67f2bae3p+0, 0x1.b5b14f08f9665p-1}, \
        {0x1.19e0119e0119ep+0, 0x1.b8e0620887309p-1}, \
        {0x1.18ab083902bdbp+0, 0x1.bc0bf57f23605p-1}, \
        {0x1.1778a191bd684p+0, 0x1.bf341114464a7p-1}, \
        {0x1.1648d50fc3201p+0, 0x1.c258bc5664829p-1}, \
        {0x1.151b9a3fdd5c9p+0, 0x1.c579febb5b657p-1}, \
        {0x1.13f0e8d344724p+0, 0x1.c897dfa0db58ep-1}, \
        {0x1.12c8b89edc0acp+0, 0x1.cbb2664ccfcf5p-1}, \
        {0x1.11a3019a74826p+0, 0x1.cec999edc5204p-1}, \
        {0x1.107fbbe011080p+0, 0x1.d1dd819b4c3f0p-1}, \
        {0x1.0f5edfab325a2p+0, 0x1.d4ee24565c62ap-1}, \
        {0x1.0e40655826011p+0, 0x1.d7fb8909b2a6cp-1}, \
        {0x1.0d24456359e3ap+0, 0x1.db05b68a2fb64p-1}, \
        {0x1.0c0a7868b4171p+0, 0x1.de0cb397338a3p-1}, \
        {0x1.0af2f722eecb5p+0, 0x1.e11086daf7497p-1}, \
        {0x1.09ddba6af8360p+0, 0x1.e41136eae553dp-1}, \
        {0x1.08cabb37565e2p+0, 0x1.e70eca47ef86fp-1}, \
        {0x1.07b9f29b8eae2p+0, 0x1.ea09475ee3c39p-1}, \
        {0x1.06ab59c7912fbp+0, 0x1.ed00b488bec24p-1}, \
        {0x1.059eea0727586p+0, 0x1.eff5180afd3e5p-1}, \
        {0x1.04949cc1664c5p+0, 0x1.f2e67817eb846p-1}, \
        {0x1.038c6b78247fcp+0, 0x1.f5d4dacef36bep-1}, \
        {0x1.02864fc7729e9p+0, 0x1.f8c0463ce8c68p-1}, \
        {0x1.0182436517a37p+0, 0x1.fba8c05c544e0p-1}, \
        {0x1.0080402010080p+0, 0x1.fe8e4f15bd1a1p-1}, \
    }
#define VNP_LP_POW_TAB \
    { \
        0x1.0000000000000p+0, \
        0x1.fc07f01fc07f0p-1, \
        0x1.f81f81f81f820p-1, \
        0x1.f44659e4a4271p-1, \
        0x1.f07c1f07c1f08p-1, \
        0x1.ecc07b301ecc0p-1, \
        0x1.e9131abf0b767p-1, \
        0x1.e573ac901e574p-1, \
        0x1.e1e1e1e1e1e1ep-1, \
        0x1.de5d6e3f8868ap-1, \
        0x1.dae6076b981dbp-1, \
        0x1.d77b654b82c34p-1, \
        0x1.d41d41d41d41dp-1, \
        0x1.d0cb58f6ec074p-1, \
        0x1.cd85689039b0bp-1, \
        0x1.ca4b3055ee191p-1, \
        0x1.c71c71c71c71cp-1, \
        0x1.c3f8f01c3f8f0p-1, \
        0x1.c0e070381c0e0p-1, \
        0x1.bdd2b899406f7p-1, \
        0x1.bacf914c1bad0p-1, \
        0x1.b7d6c3dda338bp-1, \
        0x1.b4e81b4e81b4fp-1, \
        0x1.b2036406c80d9p-1, \
        0x1.af286bca1af28p-1, \
        0x1.ac5701ac5701bp-1, \
        0x1.a98ef606a63bep-1, \
        0x1.a6d01a6d01a6dp-1, \
        0x1.a41a41a41a41ap-1, \
        0x1.a16d3f97a4b02p-1, \
        0x1.9ec8e951033d9p-1, \
        0x1.9c2d14ee4a102p-1, \
        0x1.999999999999ap-1, \
        0x1.970e4f80cb872p-1, \
        0x1.948b0fcd6e9e0p-1, \
        0x1.920fb49d0e229p-1, \
        0x1.8f9c18f9c18fap-1, \
        0x1.8d3018d3018d3p-1, \
        0x1.8acb90f6bf3aap-1, \
        0x1.886e5f0abb04ap-1, \
        0x1.8618618618618p-1, \
        0x1.83c977ab2beddp-1, \
        0x1.8181818181818p-1, \
        0x1.7f405fd017f40p-1, \
        0x1.7d05f417d05f4p-1, \
        0x1.7ad2208e0ecc3p-1, \
        0x1.78a4c8178a4c8p-1, \
        0x1.767dce434a9b1p-1, \
        0x1.745d1745d1746p-1, \
        0x1.724287f46debcp-1, \
        0x1.702e05c0b8170p-1, \
        0x1.6e1f76b4337c7p-1, \
        0x1.6c16c16c16c17p-1, \
        0x1.6a13cd1537290p-1, \
        0x1.6816816816817p-1, \
        0x1.661ec6a5122f9p-1, \
        0x1.642c8590b2164p-1, \
        0x1.623fa77016240p-1, \
        0x1.6058160581606p-1, \
        0x1.5e75bb8d015e7p-1, \
        0x1.5c9882b931057p-1, \
        0x1.5ac056b015ac0p-1, \
        0x1.58ed2308158edp-1, \
        0x1.571ed3c506b3ap-1, \
        0x1.5555555555555p-1, \
        0x1.5390948f40febp-1, \
        0x1.51d07eae2f815p-1, \
        0x1.5015015015015p-1, \
        0x1.4e5e0a72f0539p-1, \
        0x1.4cab88725af6ep-1, \
        0x1.4afd6a052bf5bp-1, \
        0x1.49539e3b2d067p-1, \
        0x1.47ae147ae147bp-1, \
        0x1.460cbc7f5cf9ap-1, \
        0x1.446f86562d9fbp-1, \
        0x1.42d6625d51f87p-1, \
        0x1.4141414141414p-1, \
        0x1.3fb013fb013fbp-1, \
        0x1.3e22cbce4a902p-1, \
        0x1.3c995a47babe7p-1, \
        0x1.3b13b13b13b14p-1, \
        0x1.3991c2c187f63p-1, \
        0x1.3813813813814p-1, \
        0x1.3698df3de0748p-1, \
        0x1.3521cfb2b78c1p-1, \
        0x1.33ae45b57bcb2p-1, \
        0x1.323e34a2b10bfp-1, \
        0x1.30d190130d190p-1, \
        0x1.2f684bda12f68p-1, \
        0x1.2e025c04b8097p-1, \
        0x1.2c9fb4d812ca0p-1, \
        0x1.2b404ad012b40p-1, \
        0x1.29e4129e4129ep-1, \
        0x1.288b01288b013p-1, \
        0x1.27350b8812735p-1, \
        0x1.25e22708092f1p-1, \
        0x1.2492492492492p-1, \
        0x1.23456789abcdfp-1, \
        0x1.21fb78121fb78p-1, \
        0x1.20b470c67c0d9p-1, \
        0x1.1f7047dc11f70p-1, \
        0x1.1e2ef3b3fb874p-1, \
        0x1.1cf06ada2811dp-1, \
        0x1.1bb4a4046ed29p-1, \
        0x1.1a7b9611a7b96p-1, \
        0x1.19453808ca29cp-1, \
        0x1.1811811811812p-1, \
        0x1.16e0689427379p-1, \
        0x1.15b1e5f75270dp-1, \
        0x1.1485f0e0acd3bp-1, \
        0x1.135c81135c811p-1, \
        0x1.12358e75d3033p-1, \
        0x1.1111111111111p-1, \
        0x1.0fef010fef011p-1, \
        0x1.0ecf56be69c90p-1, \
        0x1.0db20a88f4696p-1, \
        0x1.0c9714fbcda3bp-1, \
        0x1.0b7e6ec259dc8p-1, \
        0x1.0a6810a6810a7p-1, \
        0x1.0953f39010954p-1, \
        0x1.0842108421084p-1, \
        0x1.073260a47f7c6p-1, \
        0x1.0624dd2f1a9fcp-1, \
        0x1.05197f7d73404p-1, \
        0x1.0410410410410p-1, \
        0x1.03091b51f5e1ap-1, \
        0x1.0204081020408p-1, \
        0x1.0101010101010p-1, \
    }
static __constant__ double lp_tab_src[1 << LP_TAB_BITS][2] = VNP_LP_LOG_TAB;
static __constant__ double lp_ptab_src[1 << LP_TAB_BITS] = VNP_LP_POW_TAB;
static const double lp_ptab_host[1 << LP_TAB_BITS] = VNP_LP_POW_TAB;

}  // namespace vnp
